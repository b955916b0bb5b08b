"""Mixed strain/stress macroscopic control on the GPU (the DBFFT mixed extension the paper
relies on, Sec. 3.1) against the CPU oracle and closed forms: uniaxial stress (every
component but yy stress-free) on the fused-z grid (16^3) and on the unfused fallback
(12 x 8 x 6), a homogeneous anisotropic crystal in closed form, pure stress control,
mixed precision, and the mixed entry point with an empty mask equal to strain control."""
import numpy as np
import pytest

from oracle import OracleRVE, GrainTables, to_mandel2
from oracle.increment import from_tensor6
from synth import small_polycrystal, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu
UNIAXIAL_Y = 0b111101                # all components but yy under stress control


def _pair(w, n_inc, mask, dsig=None, precision=0):
    from paper_2304_01125_amd import RVE
    inp = make_inputs(w)
    desc = w.desc()
    gpu = RVE(desc, precision)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(w.parity().desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ds = np.zeros(6) if dsig is None else np.asarray(dsig, dtype=float)
    worst = 0.0
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=ds, stress_mask=mask)
        so = ora.step(de, inp["dt"][k], ds, mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu newton {sg['newton_iters']} krylov {sg['krylov_iters']} | oracle "
              f"newton {so['newton']} | macro stress {e:.2e} | macro strain "
              f"{np.round(sg['macro_strain'], 7).tolist()}", flush=True)
    return gpu, ora, worst


@pytest.mark.parametrize("n", [(16, 16, 16), (12, 8, 6)])
def test_uniaxial_stress_polycrystal_matches_oracle(n):
    print(f"uniaxial stress, polycrystal {n}", flush=True)
    w = small_polycrystal(n=n, n_grains=4, seed=7, amplitude=0.008).parity()
    gpu, ora, worst = _pair(w, 5, UNIAXIAL_Y)
    assert worst <= 1e-9
    compare(gpu, ora)
    ms = gpu.fields(("stress",))["stress"].mean(0)
    assert np.abs(ms[[0, 2, 3, 4, 5]]).max() <= 1e-9 * abs(ms[1])
    assert np.abs(gpu.fields(("eps_p",))["eps_p"]).max() > 1e-4      # yielded
    gpu.close()


def test_homogeneous_crystal_closed_form_and_pure_stress_control():
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=(16, 16, 16), n_grains=1, seed=4, tau_c0=1e12).parity()
    inp = make_inputs(w)
    # the macro stress is the degraded one, g(0) sigma = (1 + k_res) C eps
    C = (1.0 + w.k_res) * GrainTables(inp["quat"], w.C11, w.C12, w.C44).C[0]
    r = RVE(w.desc())
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    # uniaxial stress: E_F = -C_FF^-1 C_FP E_P
    st = r.step([0, 1e-3, 0, 0, 0, 0], 1.0, dsig6=np.zeros(6), stress_mask=UNIAXIAL_Y)
    F, P = [0, 2, 3, 4, 5], [1]
    E = np.zeros(6); E[1] = 1e-3
    E[F] = -np.linalg.solve(C[np.ix_(F, F)], C[np.ix_(F, P)] @ E[P])
    got = to_mandel2(from_tensor6(np.array(st["macro_strain"])))[0]
    print(f"  uniaxial: macro strain error {np.abs(got - E).max():.2e}", flush=True)
    assert np.abs(got - E).max() <= 1e-12 * 1e-3
    # pure stress control from there: + dsigma, strain follows C^-1
    ds = np.array([2e8, -1e8, 5e7, 3e7, -2e7, 4e7])
    st2 = r.step([0, 0, 0, 0, 0, 0], 1.0, dsig6=ds, stress_mask=63)
    sig_t = np.array(st["macro_stress"])
    dsM = to_mandel2(from_tensor6(ds))[0]
    got2 = to_mandel2(from_tensor6(np.array(st2["macro_strain"])))[0]
    print(f"  pure stress: strain error {np.abs(got2 - got - np.linalg.solve(C, dsM)).max():.2e}, "
          f"stress error {np.abs(np.array(st2['macro_stress']) - sig_t - ds).max():.2e}", flush=True)
    assert np.abs(got2 - got - np.linalg.solve(C, dsM)).max() <= 1e-12 * 1e-3
    assert np.abs(np.array(st2["macro_stress"]) - sig_t - ds).max() <= 1e-9 * np.abs(ds).max()
    r.close()


def test_mixed_precision_uniaxial_stress_within_1e4_of_oracle():
    print("mixed precision, uniaxial stress, 16^3", flush=True)
    w = small_polycrystal(n=(16, 16, 16), n_grains=4, seed=7, amplitude=0.008)
    gpu, ora, worst = _pair(w, 5, UNIAXIAL_Y, precision=1)
    assert worst <= 1e-4
    gpu.close()


def test_empty_mask_is_strain_control_bitwise():
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=(16, 16, 16), n_grains=4, seed=7, amplitude=0.008)
    inp = make_inputs(w)
    res = []
    for mixed in (False, True):
        r = RVE(w.desc())
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        for k in range(3):
            de = [0, inp["deps"][k], 0, 0, 0, 0]
            if mixed:
                from paper_2304_01125_amd.rve import rve_step_increment_mixed
                rc, _ = rve_step_increment_mixed(r.h, de, np.zeros(6), 0, inp["dt"][k])
                assert rc == 0
            else:
                r.step(de, inp["dt"][k])
        res.append(r.fields(("strain", "stress")))
        r.close()
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k
