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


def test_paper_plate_matches_stored_oracle_at_production_tolerances():
    """The paper's plate grid (256 x 256 x 1, 64 grains; Secs. 4.1-4.3) in pointwise plane
    stress under uniaxial load at the production tolerances, FP64 and mixed precision,
    against the stored oracle run (tests/golden/make_golden.py plate256): the macro stress
    and strain of every stored increment (FP64 1e-5, mixed 1e-4), sampled strain and stress
    after the first and the last, and zero out-of-plane stress.  The Newton counts differ
    (printed): the oracle solves the plane-stress condition inside every constitutive
    evaluation, the GPU condenses it in each Newton step, and both stop at the same
    solution."""
    import os
    from paper_2304_01125_amd import RVE, RVE_FP64, RVE_MIXED
    from synth import workload
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "plate256.npz"))
    last = int(ref["last"])
    w = workload("plate-256-g64")
    inp = make_inputs(w)
    idx = ref["sample"]
    for prec, bar in ((RVE_FP64, 1e-5), (RVE_MIXED, 1e-4)):
        gpu = RVE(dict(w.desc(), plane_stress=1), prec)
        gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        for k in range(last + 1):
            st = gpu.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], dsig6=np.zeros(6),
                          stress_mask=UNIAXIAL_PLATE)
            ms, me = ref["macro_stress"][k], ref["macro_strain"][k]
            es = np.abs(np.array(st["macro_stress"]) - ms).max() / np.abs(ms).max()
            ee = np.abs(np.array(st["macro_strain"]) - me).max() / np.abs(me).max()
            print(f"  precision {prec} inc {k}: newton {st['newton_iters']} (oracle "
                  f"{int(ref['newton'][k])}) macro stress {es:.2e} strain {ee:.2e}", flush=True)
            assert es <= bar and ee <= bar, (prec, k, es, ee)
            if f"inc{k}_stress" in ref.files:
                f = gpu.fields(("strain", "stress"))
                for name in ("strain", "stress"):
                    a, b = f[name][idx], ref[f"inc{k}_{name}"]
                    fe = np.linalg.norm(a - b) / np.linalg.norm(b)
                    print(f"    inc {k} {name} at {len(idx)} sampled voxels: {fe:.2e}", flush=True)
                    assert fe <= bar, (prec, k, name, fe)
        # the last Newton step condenses the linearised point; at the production stop
        # test (steps of 5e-3 of the increment) it leaves a second-order out-of-plane
        # residual (observed 2.7e-8 FP64), where the parity runs above reach 1e-10
        oop = _out_of_plane(gpu)
        print(f"    out-of-plane stress {oop:.2e} of the largest component", flush=True)
        assert oop <= 1e-6
        gpu.close()
