"""Pointwise plane stress of plates one voxel thick on the GPU (Secs. 4.1-4.3; the
out-of-plane stress zero at every voxel, the out-of-plane strain a local unknown) against
the oracle, which solves the same condition by a local iteration at every constitutive
evaluation where the GPU path condenses the linearised point inside each Newton step:
uniaxial (paper's plate loading) and strain-controlled yielding polycrystal plates in
FP64 with CG and GMRES, the mixed-precision path, a damaging plate, and the refusal of
out-of-plane macro control."""
import dataclasses

import numpy as np
import pytest

from oracle import OracleRVE
from synth import small_polycrystal, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu
UNIAXIAL_PLATE = 0b100001            # xx and xy stress free, yy strain controlled


def _pair(w, n_inc, mask, precision=0, extra=None):
    from paper_2304_01125_amd import RVE
    inp = make_inputs(w)
    desc = dict(w.desc(), plane_stress=1, **(extra or {}))
    gpu = RVE(desc, precision)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ora = OracleRVE(dict(w.parity().desc(), plane_stress=1), inp["grain"], inp["quat"],
                    inp["tau_c0"], inp["phi0"])
    worst = 0.0
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k], dsig6=np.zeros(6), stress_mask=mask)
        so = ora.step(de, inp["dt"][k], np.zeros(6), mask)
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu newton {sg['newton_iters']} krylov {sg['krylov_iters']} stag "
              f"{sg['stag_iters']} | oracle newton {so['newton']} stag {so['stag']} | macro "
              f"stress {e:.2e} | macro e_zz {sg['macro_strain'][2]:.4e}", flush=True)
    return gpu, ora, worst


def _out_of_plane(gpu):
    s = gpu.fields(("stress",))["stress"]
    return np.abs(s[:, 2:5]).max() / np.abs(s).max()


@pytest.mark.parametrize("krylov", [0, 1])
def test_uniaxial_polycrystal_plate_matches_oracle(krylov):
    print(f"plate 16x12x1, 5 grains, uniaxial, krylov {krylov}", flush=True)
    w = small_polycrystal(n=(16, 12, 1), n_grains=5, seed=3, amplitude=0.008).parity()
    gpu, ora, worst = _pair(w, 5, UNIAXIAL_PLATE, extra=dict(krylov=krylov, gmres_restart=30))
    assert worst <= 1e-9
    compare(gpu, ora)
    assert _out_of_plane(gpu) <= 1e-10
    assert np.abs(gpu.fields(("eps_p",))["eps_p"]).max() > 1e-4      # yielded
    gpu.close()


def test_strain_controlled_plate_on_an_unfused_grid_matches_oracle():
    print("plate 12x18x1, 4 grains, strain control", flush=True)
    w = small_polycrystal(n=(12, 18, 1), n_grains=4, seed=9, amplitude=0.008).parity()
    gpu, ora, worst = _pair(w, 4, 0)
    assert worst <= 1e-9
    compare(gpu, ora)
    assert _out_of_plane(gpu) <= 1e-10
    gpu.close()


def test_mixed_precision_plate_within_1e4_of_oracle():
    from paper_2304_01125_amd import RVE_MIXED
    print("plate 16x12x1 mixed precision", flush=True)
    w = small_polycrystal(n=(16, 12, 1), n_grains=5, seed=3, amplitude=0.008)
    w = dataclasses.replace(w, tol_newton=1e-6, tol_lin=1e-7, tol_stag=1e-6)
    gpu, ora, worst = _pair(w, 5, UNIAXIAL_PLATE, precision=RVE_MIXED)
    assert worst <= 1e-4
    assert _out_of_plane(gpu) <= 1e-5
    gpu.close()


def test_damaging_plate_matches_oracle():
    print("plate 16x16x1, 3 grains, damage active", flush=True)
    w = dataclasses.replace(small_polycrystal(n=(16, 16, 1), n_grains=3, seed=5),
                            G_crit=0.004, Gc=100.0, amplitude=0.006).parity()
    gpu, ora, worst = _pair(w, 6, UNIAXIAL_PLATE)
    assert ora.trig.sum() > 20 and ora.phi.max() > 0.005
    assert worst <= 1e-9
    compare(gpu, ora)
    assert _out_of_plane(gpu) <= 1e-10
    gpu.close()


def test_out_of_plane_macro_control_is_refused():
    from paper_2304_01125_amd import RVE, RveError, RVE_E_ARG
    w = small_polycrystal(n=(8, 6, 1), n_grains=2, seed=1)
    inp = make_inputs(w)
    gpu = RVE(dict(w.desc(), plane_stress=1))
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for de, mask in (([0, 1e-4, 1e-4, 0, 0, 0], 0), ([0, 1e-4, 0, 0, 1e-5, 0], 0),
                     ([0, 1e-4, 0, 0, 0, 0], 0b000100)):
        with pytest.raises(RveError) as e:
            gpu.step(de, 1.0, dsig6=np.zeros(6), stress_mask=mask)
        assert e.value.code == RVE_E_ARG
    st = gpu.step([0, 1e-4, 0, 0, 0, 0], 1.0, dsig6=np.zeros(6), stress_mask=UNIAXIAL_PLATE)
    assert abs(st["macro_strain"][1] - 1e-4) <= 1e-15
    gpu.close()
