"""The options together against the CPU oracle at tight tolerances: the paper's thermally
activated flow rule with Taylor hardening, the rotated-scheme derivative and uniaxial-stress
control (CG) in one run, and the same material and derivative under strain control with the
paper's GMRES(30) solver, through yielding increments of a 12 x 8 x 6 polycrystal."""
import numpy as np
import pytest

from oracle import OracleRVE
from synth import small_polycrystal, make_inputs, cmsx4
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("krylov,mask", [(0, 0b111101), (1, 0)])
def test_flow_rule_rotated_scheme_and_control_together(krylov, mask):
    from paper_2304_01125_amd import RVE
    print(f"cmsx4 material, rotated scheme, krylov {krylov}, stress mask {mask}", flush=True)
    w = small_polycrystal(n=(12, 8, 6), n_grains=4, seed=7, cycles=1, incs_per_cycle=20,
                          **cmsx4()).parity()
    d = dict(w.desc(), scheme=1)
    inp = make_inputs(w)
    gpu = RVE(dict(d, krylov=krylov, max_krylov=20000))
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(d, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(5):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=mask)
        so = ora.step(de, inp["dt"][k], np.zeros(6), mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        print(f"  inc {k}: newton {sg['newton_iters']} (oracle {so['newton']}) krylov "
              f"{sg['krylov_iters']} macro stress {e:.2e}", flush=True)
        assert e <= 1e-9
    compare(gpu, ora)
    assert np.abs(gpu.fields(("eps_p",))["eps_p"]).max() > 1e-3
    gpu.close()
