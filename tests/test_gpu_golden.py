"""Parity of the GPU path with stored oracle results at the workloads' full sizes.

The expected values were written by tests/golden/make_golden.py, which calls only the
CPU oracle (tight tolerances): the notched single crystal on 16^3 up to and including
the increment where the damage first jumps by more than 0.5, and sampled voxels of the
first increments of the 64^3 Voronoi polycrystal."""
import os

import numpy as np
import pytest

from synth import workload, make_inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _check(f, ref, prefix, tol=1e-9, tol_phi=1e-8, idx=None):
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    errs = {k: rel_l2(sel(f[k]), ref[f"{prefix}_{k}"]) for k in ("strain", "stress", "gs", "wp")}
    errs["damage"] = np.abs(sel(f["damage"]) - ref[f"{prefix}_damage"]).max()
    print(f"  {prefix}:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["strain"] <= tol and errs["stress"] <= tol
    assert errs["damage"] <= tol_phi
    assert errs["gs"] <= 1e-8 and errs["wp"] <= 1e-8


def test_notched_crystal_16_matches_stored_oracle():
    from paper_2304_01125_amd import RVE
    ref = np.load(os.path.join(GOLDEN, "notched16.npz"))
    last, jump = int(ref["last"]), int(ref["jump_inc"])
    w = workload("notched-crystal-16").parity()
    inp = make_inputs(w)
    r = RVE(w.desc())
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    names = ("strain", "stress", "damage", "gs", "wp")
    for k in range(jump + 1):
        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        print(f"  inc {k}: newton {st['newton_iters']} krylov {st['krylov_iters']} "
              f"stag {st['stag_iters']} max phi (slip) {st['max_phi_slip']:.4f}", flush=True)
        if k <= last:
            ms = np.array(st["macro_stress"])
            assert np.abs(ms - ref["macro_stress"][k]).max() <= 1e-9 * np.abs(ref["macro_stress"][k]).max()
        if f"inc{k}_strain" in ref.files:
            _check(r.fields(names), ref, f"inc{k}")
    # the increment of the first damage jump (> 0.5): still a unique converged state
    _check(r.fields(names), ref, "jump", tol=1e-8, tol_phi=1e-7)
    r.close()


def test_voronoi_64_sampled_voxels_match_stored_oracle():
    """Config 1 up to damage initiation: the macro stress, the number of triggered voxels
    and the maximum damage of every increment, and the sampled fields after increment 1
    and the last two increments (the first voxel triggered, then damage active: about 50
    alternating passes), against the stored oracle run."""
    from paper_2304_01125_amd import RVE
    ref = np.load(os.path.join(GOLDEN, "voronoi64.npz"))
    idx = ref["sample"]
    w = workload("voronoi-64-g64").parity()
    assert w.G_crit == float(ref["G_crit"])
    inp = make_inputs(w)
    r = RVE(w.desc())
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    last = int(ref["last"])
    for k in range(last + 1):
        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        print(f"  inc {k}: newton {st['newton_iters']} krylov {st['krylov_iters']} stag "
              f"{st['stag_iters']} triggered {st['n_triggered']:.0f} max phi "
              f"{st['max_phi']:.3e} (oracle {ref['n_trig'][k]}, {ref['max_phi'][k]:.3e})",
              flush=True)
        ms = np.array(st["macro_stress"])
        assert np.abs(ms - ref["macro_stress"][k]).max() <= 1e-9 * np.abs(ref["macro_stress"][k]).max()
        assert st["n_triggered"] == ref["n_trig"][k]
        assert abs(st["max_phi"] - ref["max_phi"][k]) <= 1e-8
        if f"inc{k}_strain" in ref.files:
            f = r.fields(("strain", "stress", "damage", "gs", "wp", "h", "wcrit", "trig"))
            _check(f, ref, f"inc{k}", idx=idx)
            for name in ("h", "wcrit"):
                a, b = f[name][idx], ref[f"inc{k}_{name}"]
                e = rel_l2(a, b) if np.linalg.norm(b) > 0 else np.abs(a).max()
                assert e <= 1e-8, (name, e)
            assert np.array_equal(f["trig"][idx], ref[f"inc{k}_trig"])
    # damage initiated from the stored energy within the stored increments
    assert ref["max_phi"][last] > 0.0 and ref["n_trig"][last] > 0
    r.close()
