"""The rotated-scheme discrete derivative on the GPU (Sec. 3.1's discrete-derivative remedy
for Gibbs oscillations) against the CPU oracle: the preconditioned operator on fused-z and
unfused grids, whole increments of a yielding polycrystal (FP64 and mixed precision, with
strain and with uniaxial-stress control), and the 128^3 benchmark increment (equilibrium
under the rotated divergence, return map at sampled voxels)."""
import numpy as np
import pytest

from oracle import Grid, OracleRVE, GrainTables, return_map, to_mandel2, from_mandel2
from oracle.crystal import from_mandel4
from oracle.increment import from_tensor6
from synth import small_polycrystal, workload, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [(32, 8, 128), (16, 16, 16), (12, 8, 6), (18, 64, 64),
                               (128, 2, 256)])
@pytest.mark.parametrize("prec", [0, 1])
def test_operator_matches_oracle(n, prec):
    from paper_2304_01125_amd import RVE
    print(f"rotated operator {n} precision {prec}", flush=True)
    w = small_polycrystal(n=n, n_grains=4, seed=3)
    d = dict(w.desc(), scheme=1)
    inp = make_inputs(w)
    r = RVE(d, prec)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    rng = np.random.default_rng(0)
    M = w.nvox
    eps = rng.uniform(-4e-3, 4e-3, (M, 6))
    eps[:, 1] += 8e-3
    _, gk = r.constitutive(eps, 1.0)
    g = Grid(n, w.h, scheme=1)
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


def _pair(n, precision=0, mask=0, n_inc=4):
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=n, n_grains=4, seed=7, amplitude=0.008)
    wp = w.parity()
    inp = make_inputs(w)
    gpu = RVE(dict((wp if precision == 0 else w).desc(), scheme=1), precision)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(dict(wp.desc(), scheme=1), inp["grain"], inp["quat"], inp["tau_c0"],
                    inp["phi0"])
    worst = 0.0
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=mask)
        so = ora.step(de, inp["dt"][k], np.zeros(6), mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu newton {sg['newton_iters']} krylov {sg['krylov_iters']} | oracle "
              f"newton {so['newton']} | macro stress {e:.2e}", flush=True)
    return gpu, ora, worst


@pytest.mark.parametrize("n", [(16, 16, 16), (12, 8, 6)])
@pytest.mark.parametrize("mask", [0, 0b111101])
def test_increments_match_oracle(n, mask):
    print(f"rotated scheme increments {n} stress mask {mask}", flush=True)
    gpu, ora, worst = _pair(n, 0, mask)
    assert worst <= 1e-9
    compare(gpu, ora)
    gpu.close()


def test_mixed_precision_within_1e4_of_oracle():
    gpu, ora, worst = _pair((16, 16, 16), 1, 0)
    assert worst <= 1e-4
    gpu.close()


def test_first_increment_at_full_size():
    from paper_2304_01125_amd import RVE, RVE_FP64
    w = workload("laguerre-128-g512").parity()
    inp = make_inputs(w)
    r = RVE(dict(w.desc(), scheme=1), RVE_FP64)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    st = r.step([0, inp["deps"][0], 0, 0, 0, 0], inp["dt"][0])
    print(f"  rotated 128^3: newton {st['newton_iters']} krylov {st['krylov_iters']}", flush=True)
    f = r.fields(("strain", "stress", "stress_eff"))
    r.close()
    assert np.abs(f["strain"].mean(0)[1] - inp["deps"][0]) <= 1e-15
    g = Grid(w.n, w.h, scheme=1)
    sh = g.fft(g.to_grid(from_tensor6(f["stress"])))
    div = np.abs(g.div_hat(sh)).max() / (np.abs(sh).max() * np.abs(g.k).max())
    idx = np.random.default_rng(13).choice(w.nvox, 4096, replace=False)
    tab = GrainTables(inp["quat"], w.C11, w.C12, w.C44)
    gid = inp["grain"][idx]
    epsM = to_mandel2(from_tensor6(f["strain"][idx]))
    sig, _, _, _ = return_map(epsM, np.zeros_like(epsM), np.asarray(inp["tau_c0"])[gid],
                              inp["dt"][0], tab.C[gid], tab.S[gid], tab.P[gid], w.gdot0, w.n_exp)
    e_sig = np.linalg.norm(to_mandel2(from_tensor6(f["stress_eff"][idx])) - sig) / \
        np.linalg.norm(sig)
    print(f"  equilibrium (rotated divergence) {div:.2e}; sampled stress {e_sig:.2e}", flush=True)
    assert div <= 1e-9 and e_sig <= 1e-10
