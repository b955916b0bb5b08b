"""GPU building blocks against the CPU oracle, through the C ABI diagnostics:
3-D real FFT (Sec. 3.1), the per-voxel return map and tangent (Sec. 2.1), and the
preconditioned linearised equilibrium operator (eqs. newton, precf, avstiff)."""
import numpy as np
import pytest

from oracle import Grid, GrainTables, return_map, to_mandel2, from_mandel2
from oracle.crystal import from_mandel4
from oracle.increment import tensor6, from_tensor6
from synth import small_polycrystal, make_inputs

pytestmark = pytest.mark.gpu

SIZES = [(4, 4, 4), (3, 3, 3), (6, 4, 3), (16, 16, 16), (48, 32, 12), (12, 18, 9), (64, 8, 4),
         (128, 128, 4), (32, 8, 128), (96, 48, 96), (256, 256, 2), (18, 64, 64)]


def _rve(n, precision=0, n_grains=4, seed=3):
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=n, n_grains=n_grains, seed=seed)
    return w, RVE(w.desc(), precision)


def _half(g, F):
    """Oracle full spectrum (N1,N2,N3,...) -> half spectrum in the library's bin order."""
    n1h = g.n[0] // 2 + 1
    H = F[:n1h]
    rest = H.shape[3:]
    return np.moveaxis(H, (0, 1, 2), (2, 1, 0)).reshape((-1,) + rest)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("prec", [0, 1])
def test_rfft_matches_oracle(n, prec):
    print(f"rfft n={n} precision={prec}", flush=True)
    w, r = _rve(n, prec)
    g = Grid(n, w.h)
    rng = np.random.default_rng(sum(n))
    f = rng.standard_normal((3, g.M))
    spec = r.rfft(f, 3)
    tol = 1e-13 if prec == 0 else 2e-6
    for c in range(3):
        ref = _half(g, g.fft(g.to_grid(f[c])))
        err = np.abs(spec[c] - ref).max() / np.abs(ref).max()
        assert err <= tol, (c, err)
    back = r.irfft(spec, 3)
    assert np.abs(back - f).max() <= (1e-14 if prec == 0 else 2e-6) * 10
    r.close()


def _constitutive_case(n=(8, 6, 4), prec=0, amp=4e-3, seed=0):
    w, r = _rve(n, prec)
    inp = make_inputs(w)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    rng = np.random.default_rng(seed)
    M = int(np.prod(n))
    eps = rng.uniform(-amp, amp, (M, 6))
    eps[:, 1] += 2 * amp
    return w, r, inp, eps


def test_constitutive_matches_oracle():
    print("constitutive 8x6x4", flush=True)
    w, r, inp, eps = _constitutive_case()
    sig_g, gk_g = r.constitutive(eps, 1.0)
    t = GrainTables(inp["quat"], w.C11, w.C12, w.C44)
    gid = inp["grain"]
    g = np.full(len(gid), w.tau_c0)
    sig_o, dg, K, _ = return_map(to_mandel2(from_tensor6(eps)), np.zeros((len(gid), 6)), g, 1.0,
                                 t.C[gid], t.S[gid], t.P[gid], w.gdot0, w.n_exp)
    sig_o6 = tensor6(from_mandel2(sig_o))
    assert np.abs(dg).max() > 1e-3                         # genuinely plastic voxels
    err = np.abs(sig_g - sig_o6).max() / np.abs(sig_o6).max()
    assert err <= 1e-12, err
    iu = np.triu_indices(6)
    Ko = (1.0 + w.k_res) * K[:, iu[0], iu[1]]              # phi = 0: g = 1 + k
    errk = np.abs(gk_g - Ko).max() / np.abs(Ko).max()
    assert errk <= 1e-10, errk
    r.close()


def test_operator_matches_oracle_and_is_identity_for_homogeneous_tangent():
    print("operator 8x6x4", flush=True)
    w, r, inp, eps = _constitutive_case()
    _, gk = r.constitutive(eps, 1.0)
    n = w.n
    g = Grid(n, w.h)
    iu = np.triu_indices(6)
    Km = np.zeros((g.M, 6, 6))
    Km[:, iu[0], iu[1]] = gk
    Km[:, iu[1], iu[0]] = gk
    rng = np.random.default_rng(1)
    u = rng.standard_normal((g.M, 3)) * 1e-9
    v = r.operator(u)
    Ainv = g.acoustic_inverse(from_mandel4(Km.mean(0)))
    Kg = g.to_grid(Km)
    ug = g.to_grid(u)
    de = g.ifft(g.sym_grad_hat(g.fft(ug)))
    ds = from_mandel2(np.einsum("...ij,...j->...i", Kg, to_mandel2(de)))
    ref = g.ifft(np.einsum("...ik,...k->...i", Ainv, -g.div_hat(g.fft(ds))))
    ref = g.to_flat(ref)
    err = np.abs(v - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err
    r.close()


# fused z passes with work-unit counts that are multiples of 8 (XCD-contiguous block
# order) and not (plain order: 16x12x16, 48x12x48), unfused grids, both precisions; every
# column length of the fused z passes (16, 32, 48, 64, 96, 128, 256) and the row tangent
# pass at rows of 96, 128 and 256 (256-thread blocks); 64-bin tiles of the FP32 inverse z
# pass (rows of 128 and 256); the wide tiles of 256-point columns (one block per CU: 32- and
# 16-bin FP64, 64- and 32-bin FP32 tiles) on rows of 128
FUSED = [(32, 8, 128), (16, 16, 16), (16, 12, 16), (48, 12, 48), (64, 64, 64), (16, 8, 32),
         (16, 8, 96), (96, 8, 96), (16, 4, 256), (256, 8, 16), (128, 6, 16), (128, 2, 256)]
# (128, 9, 3): the unfused path on rows of 128


@pytest.mark.parametrize("n", FUSED + [(12, 8, 6), (128, 9, 3)])
@pytest.mark.parametrize("prec", [0, 1])
def test_operator_shapes_match_oracle(n, prec):
    from paper_2304_01125_amd import RveError
    print(f"operator {n} precision {prec}", flush=True)
    w, r = _rve(n, prec)
    # the grids listed as fused do take the fused z passes (zero launches: a query)
    try:
        r.launch_pass(8, 0)
        fused = True
    except RveError:
        fused = False
    assert fused == (n in FUSED), (n, fused)
    inp = make_inputs(w)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    rng = np.random.default_rng(0)
    M = w.nvox
    eps = rng.uniform(-4e-3, 4e-3, (M, 6))
    eps[:, 1] += 8e-3
    _, gk = r.constitutive(eps, 1.0)
    g = Grid(n, w.h)
    iu = np.triu_indices(6)
    Km = np.zeros((M, 6, 6))
    Km[:, iu[0], iu[1]] = gk
    Km[:, iu[1], iu[0]] = gk
    u = rng.standard_normal((M, 3)) * 1e-9
    v = r.operator(u)
    r.close()
    Ainv = g.acoustic_inverse(from_mandel4(Km.mean(0)))
    Kg = g.to_grid(Km)
    de = g.ifft(g.sym_grad_hat(g.fft(g.to_grid(u))))
    ds = from_mandel2(np.einsum("...ij,...j->...i", Kg, to_mandel2(de)))
    ref = g.to_flat(g.ifft(np.einsum("...ik,...k->...i", Ainv, -g.div_hat(g.fft(ds)))))
    err = np.abs(v - ref).max() / np.abs(ref).max()
    print(f"  error {err:.2e}", flush=True)
    assert err <= (1e-12 if prec == 0 else 2e-5)
