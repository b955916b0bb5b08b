"""Edge cases of the GPU path against the CPU oracle: the maximum axis length (512) and
single-voxel axes in the FFTs and the operator; a single-voxel RVE (one material point); a
one-voxel-thick plate under uniaxial stress with soft free-surface buffer columns (pre-set
damage, stiffness k C) as in the paper's plate setups."""
import numpy as np
import pytest

from oracle import Grid, OracleRVE, from_mandel2, to_mandel2
from oracle.crystal import from_mandel4
from synth import small_polycrystal, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu


def _half(g, F):
    n1h = g.n[0] // 2 + 1
    H = F[:n1h]
    return np.moveaxis(H, (0, 1, 2), (2, 1, 0)).reshape((-1,) + H.shape[3:])


@pytest.mark.parametrize("n", [(512, 2, 2), (2, 512, 2), (2, 2, 512), (1, 1, 1), (1, 9, 1),
                               (3, 1, 4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_rfft_at_extreme_axis_lengths(n, prec):
    from paper_2304_01125_amd import RVE
    print(f"rfft {n} precision {prec}", flush=True)
    w = small_polycrystal(n=n, n_grains=1, seed=1)
    r = RVE(w.desc(), prec)
    g = Grid(n, w.h)
    f = np.random.default_rng(sum(n)).standard_normal((2, g.M))
    spec = r.rfft(f, 2)
    tol = 1e-13 if prec == 0 else 3e-6
    for c in range(2):
        ref = _half(g, g.fft(g.to_grid(f[c])))
        assert np.abs(spec[c] - ref).max() <= tol * np.abs(ref).max()
    assert np.abs(r.irfft(spec, 2) - f).max() <= 10 * tol
    r.close()


@pytest.mark.parametrize("n", [(512, 4, 2), (2, 4, 512), (4, 512, 2)])
def test_operator_at_maximum_axis_length(n):
    from paper_2304_01125_amd import RVE
    print(f"operator {n}", flush=True)
    w = small_polycrystal(n=n, n_grains=4, seed=3)
    inp = make_inputs(w)
    r = RVE(w.desc())
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    rng = np.random.default_rng(2)
    M = w.nvox
    eps = rng.uniform(-4e-3, 4e-3, (M, 6))
    eps[:, 1] += 8e-3
    _, gk = r.constitutive(eps, 1.0)
    u = rng.standard_normal((M, 3)) * 1e-9
    v = r.operator(u)
    r.close()
    g = Grid(n, w.h)
    iu = np.triu_indices(6)
    Km = np.zeros((M, 6, 6))
    Km[:, iu[0], iu[1]] = gk
    Km[:, iu[1], iu[0]] = gk
    Ainv = g.acoustic_inverse(from_mandel4(Km.mean(0)))
    de = g.ifft(g.sym_grad_hat(g.fft(g.to_grid(u))))
    ds = from_mandel2(np.einsum("...ij,...j->...i", g.to_grid(Km), to_mandel2(de)))
    ref = g.to_flat(g.ifft(np.einsum("...ik,...k->...i", Ainv, -g.div_hat(g.fft(ds)))))
    err = np.abs(v - ref).max() / np.abs(ref).max()
    print(f"  error {err:.2e}", flush=True)
    assert err <= 1e-12


def _pair(w, n_inc, mask=0):
    from paper_2304_01125_amd import RVE
    inp = make_inputs(w)
    gpu = RVE(w.desc())
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=mask)
        so = ora.step(de, inp["dt"][k], np.zeros(6), mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        print(f"  inc {k}: newton {sg['newton_iters']} krylov {sg['krylov_iters']} "
              f"(oracle newton {so['newton']}) macro stress {e:.2e}", flush=True)
        assert e <= 1e-9
    return gpu, ora


@pytest.mark.parametrize("mask", [0, 0b111101])
def test_single_voxel_is_one_material_point(mask):
    w = small_polycrystal(n=(1, 1, 1), n_grains=1, seed=2, amplitude=0.008).parity()
    gpu, ora = _pair(w, 6, mask)
    compare(gpu, ora)
    gpu.close()


def test_thin_plate_with_soft_surface_buffers_under_uniaxial_stress():
    # 24 x 8 x 1 voxels, 6 grains; columns x = 0, 1 are a soft buffer (phi0 = 1: stiffness
    # k C, no slip); yy strain imposed, every other macro stress held at zero
    w = small_polycrystal(n=(24, 8, 1), n_grains=6, seed=4, amplitude=0.008).parity()
    inp = make_inputs(w)
    phi0 = np.zeros(w.nvox)
    x = np.arange(w.nvox) % w.n[0]
    phi0[x < 2] = 1.0
    from paper_2304_01125_amd import RVE
    gpu = RVE(w.desc())
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], phi0)
    ora = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], phi0)
    for k in range(4):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=0b111101)
        so = ora.step(de, inp["dt"][k], np.zeros(6), 0b111101)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        print(f"  inc {k}: newton {sg['newton_iters']} krylov {sg['krylov_iters']} "
              f"macro stress {e:.2e}", flush=True)
        assert e <= 1e-9
    compare(gpu, ora)
    s = gpu.fields(("stress",))["stress"]
    # the buffer carries (almost) no stress
    assert np.abs(s[x < 2]).max() <= 1e-3 * np.abs(s[x >= 2]).max()
    gpu.close()
