"""Finite-strain kinematics on the GPU against the finite-strain oracle (Sec. 2.1: F = Fe Fp,
first Piola-Kirchhoff stress; Sec. 3.1 eqs. fdef, newton, precf with the 9-component
gradient and the 9 x 9 tangent; eq. decMiehe with the log elastic strain), through the C
ABI: the per-voxel return map and consistent tangent, whole increments of yielding and of
damaging polycrystals at tight tolerances, and the 16^3 polycrystal against stored oracle
results."""
import dataclasses
import os

import numpy as np
import pytest

from oracle import GrainTables, PowerLaw
from oracle.finite import OracleFiniteRVE, fs_return_map, fs_tangent
from synth import small_polycrystal, make_inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _desc(w):
    return dict(w.desc(), kinematics=1, krylov=1, gmres_restart=30)


def _gpu(w):
    from paper_2304_01125_amd import RVE
    inp = make_inputs(w)
    r = RVE(_desc(w))
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    return inp, r


def test_constitutive_and_tangent_match_oracle():
    print("finite-strain constitutive 8x6x4", flush=True)
    w = small_polycrystal(n=(8, 6, 4), n_grains=4, seed=3)
    inp, r = _gpu(w)
    M = w.nvox
    rng = np.random.default_rng(5)
    F = np.eye(3) + rng.uniform(-5e-3, 5e-3, (M, 3, 3))
    F[:, 1, 1] += 4e-3
    P_g, K_g = r.constitutive_finite(F.reshape(M, 9), 1.0)
    r.close()
    tab = GrainTables(inp["quat"], w.C11, w.C12, w.C44)
    gid = np.asarray(inp["grain"], dtype=np.int64)
    o = fs_return_map(F, np.tile(np.eye(3), (M, 1, 1)), np.asarray(inp["tau_c0"])[gid], 1.0, tab,
                      gid, PowerLaw(w.gdot0, w.n_exp))
    K_o = (1.0 + w.k_res) * fs_tangent(F, o).reshape(M, 9, 9)
    assert np.abs(o["dgam"]).max() > 1e-4                     # genuinely plastic voxels
    eP = np.abs(P_g - o["P"].reshape(M, 9)).max() / np.abs(o["P"]).max()
    eK = np.abs(K_g - K_o).max() / np.abs(K_o).max()
    print(f"  P {eP:.2e}, K {eK:.2e}", flush=True)
    assert eP <= 1e-12 and eK <= 1e-10


def _compare(r, o, tol_field=1e-9, tol_phi=1e-8):
    f = r.fields(("defgrad", "pk1", "fp", "damage", "gs", "wp", "h", "wcrit", "trig", "rho_ssd",
                  "rho_gnd", "g"))
    ref = o.fields()
    errs = {k: rel_l2(f[k], ref[k]) for k in ("defgrad", "pk1", "fp", "gs", "wp", "rho_ssd")}
    errs["damage"] = np.abs(f["damage"] - ref["damage"]).max()
    for k in ("h", "wcrit", "rho_gnd"):
        errs[k] = rel_l2(f[k], ref[k]) if np.linalg.norm(ref[k]) > 0 else np.abs(f[k]).max()
    errs["trig_mismatch"] = float(np.count_nonzero(f["trig"] != ref["trig"]))
    print("  errors:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["defgrad"] <= tol_field and errs["pk1"] <= tol_field
    assert errs["damage"] <= tol_phi and errs["trig_mismatch"] == 0
    for k in ("fp", "gs", "wp", "rho_ssd", "h", "wcrit", "rho_gnd"):
        assert errs[k] <= 1e-8, (k, errs[k])


def _pair(w, n_inc):
    inp, r = _gpu(w)
    o = OracleFiniteRVE(_desc(w), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(n_inc):
        dF = np.zeros(9)
        dF[4] = inp["deps"][k]
        sg = r.step_finite(dF, inp["dt"][k])
        so = o.step(dF, inp["dt"][k])
        e = np.abs(np.array(sg["macro_pk1"]) - so["macro_stress"]).max() / np.abs(so["macro_stress"]).max()
        print(f"  inc {k}: gpu newton {sg['newton_iters']} krylov {sg['krylov_iters']} stag "
              f"{sg['stag_iters']} pf {sg['pf_iters']} | oracle newton {so['newton']} stag "
              f"{so['stag']} | macro P {e:.2e}", flush=True)
        assert e <= 1e-9
        # the mean of N values near 1, summed in different orders: rounding only
        assert np.abs(np.array(sg["macro_defgrad"]) - so["macro_defgrad"]).max() <= 1e-14
    return r, o


def test_yielding_increments_match_oracle():
    print("finite strain 12x8x6, 4 grains, 4 yielding increments", flush=True)
    w = small_polycrystal(n=(12, 8, 6), n_grains=4, seed=7).parity()
    r, o = _pair(w, 4)
    assert np.abs(o.Wp).max() > 1e4                          # kJ/m^3 of plastic work
    _compare(r, o)
    r.close()


def test_damaging_increments_match_oracle():
    print("finite strain 8x8x8, 3 grains, damage active", flush=True)
    w = dataclasses.replace(small_polycrystal(n=(8, 8, 8), n_grains=3, seed=5), G_crit=0.004,
                            Gc=100.0, amplitude=0.006).parity()
    r, o = _pair(w, 6)
    assert o.trig.sum() > 100 and o.phi.max() > 0.005 and o.history[-1]["stag"] > 3
    _compare(r, o)
    r.close()


def test_finite16_matches_stored_oracle():
    """The 16^3 eight-grain polycrystal (tests/golden/make_golden.py finite16)."""
    import sys
    sys.path.insert(0, GOLDEN)
    from make_golden import finite_workload, FIELDS_FINITE
    ref = np.load(os.path.join(GOLDEN, "finite16.npz"))
    w = finite_workload()
    inp, r = _gpu(w)
    for k in range(int(ref["last"]) + 1):
        dF = np.zeros(9)
        dF[4] = inp["deps"][k]
        st = r.step_finite(dF, inp["dt"][k])
        ms = np.array(st["macro_pk1"])
        e = np.abs(ms - ref["macro_pk1"][k]).max() / np.abs(ref["macro_pk1"][k]).max()
        print(f"  inc {k}: newton {st['newton_iters']} (oracle {int(ref['newton'][k])}) "
              f"krylov {st['krylov_iters']} macro P {e:.2e}", flush=True)
        assert e <= 1e-9
        if f"inc{k}_defgrad" in ref.files:
            f = r.fields(FIELDS_FINITE)
            errs = {n: rel_l2(f[n], ref[f"inc{k}_{n}"]) for n in FIELDS_FINITE if n != "damage"}
            errs["damage"] = np.abs(f["damage"] - ref[f"inc{k}_damage"]).max()
            print(f"  inc {k} fields:", {n: f"{v:.1e}" for n, v in errs.items()}, flush=True)
            assert errs["defgrad"] <= 1e-9 and errs["pk1"] <= 1e-9 and errs["damage"] <= 1e-8
            for n in ("fp", "gs", "wp", "rho_ssd", "rho_gnd", "g", "h"):
                assert errs[n] <= 1e-8, (n, errs[n])
    r.close()


def test_small_and_finite_entry_points_refuse_each_other():
    from paper_2304_01125_amd import RVE, RveError, RVE_E_ARG
    w = small_polycrystal(n=(8, 6, 4), n_grains=2, seed=1)
    inp, r = _gpu(w)
    with pytest.raises(RveError) as e:
        r.step([0, 1e-3, 0, 0, 0, 0], 1.0)
    assert e.value.code == RVE_E_ARG
    with pytest.raises(RveError) as e:
        r.fields(("strain",))
    assert e.value.code == RVE_E_ARG
    r.close()
    s = RVE(w.desc())
    s.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    with pytest.raises(RveError) as e:
        s.step_finite(np.zeros(9), 1.0)
    assert e.value.code == RVE_E_ARG
    with pytest.raises(RveError) as e:
        s.fields(("defgrad",))
    assert e.value.code == RVE_E_ARG
    s.close()
