"""The restarted GMRES(m) option of the momentum Krylov solve (the paper's solver, eq.
newton with the preconditioner of eqs. precf and avstiff) against the CPU oracle: the
linearised operator is symmetric positive definite, so GMRES and CG reach the same Newton
corrections and the same increments (tight tolerances); mixed precision within 1e-4; a
restart length of 1 (steepest-descent-like restarts) still converges; mixed macroscopic
control (uniaxial stress: the stress-controlled macro strains ride in the zero bin of the
Krylov vectors, with the macro block of the preconditioner) gives the oracle's increments
with GMRES as with CG."""
import numpy as np
import pytest

from oracle import OracleRVE
from synth import small_polycrystal, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu


def _pair(n, precision=0, restart=30, n_inc=4, parity=True):
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=n, n_grains=4, seed=7, amplitude=0.008)
    wp = w.parity()
    inp = make_inputs(w)
    gpu = RVE(dict((wp if parity else w).desc(), krylov=1, gmres_restart=restart,
                   max_krylov=20000), precision)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(wp.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    worst = 0.0
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k])
        so = ora.step(de, inp["dt"][k])
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu newton {sg['newton_iters']} gmres {sg['krylov_iters']} | oracle "
              f"newton {so['newton']} | macro stress {e:.2e}", flush=True)
    return gpu, ora, worst


@pytest.mark.parametrize("n", [(16, 16, 16), (12, 8, 6)])
def test_gmres_increments_match_oracle(n):
    print(f"GMRES(30) increments {n}", flush=True)
    gpu, ora, worst = _pair(n)
    assert worst <= 1e-9
    compare(gpu, ora)
    gpu.close()


def test_gmres_restart_one_converges_to_the_same_increment():
    gpu, ora, worst = _pair((12, 8, 6), restart=1, n_inc=2)
    assert worst <= 1e-9
    gpu.close()


def test_gmres_mixed_precision_within_1e4_of_oracle():
    gpu, ora, worst = _pair((16, 16, 16), precision=1, parity=False)
    assert worst <= 1e-4
    gpu.close()


@pytest.mark.parametrize("n", [(16, 16, 16), (12, 8, 6)])
def test_gmres_under_uniaxial_stress_matches_oracle(n):
    from paper_2304_01125_amd import RVE
    print(f"GMRES(30) under uniaxial stress {n}", flush=True)
    w = small_polycrystal(n=n, n_grains=4, seed=7, amplitude=0.008).parity()
    inp = make_inputs(w)
    gpu = RVE(dict(w.desc(), krylov=1, gmres_restart=30, max_krylov=20000), 0)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    mask = 0b111101
    worst = 0.0
    for k in range(5):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=mask)
        so = ora.step(de, inp["dt"][k], np.zeros(6), mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu newton {sg['newton_iters']} gmres {sg['krylov_iters']} | oracle "
              f"newton {so['newton']} | macro stress {e:.2e}", flush=True)
        assert sg["newton_iters"] == so["newton"]
    assert worst <= 1e-9
    compare(gpu, ora)
    ms = gpu.fields(("stress",))["stress"].mean(0)
    assert np.abs(ms[[0, 2, 3, 4, 5]]).max() <= 1e-9 * abs(ms[1])
    gpu.close()
