"""The phase-field option that holds the pre-set crack at phi = 1 as a Dirichlet condition
(the geometric crack of the numerical examples, Secs. 4.1 and 4.5, read as a boundary value
of the damage) on the GPU against the CPU oracle: whole increments of a yielding,
damaging three-grain polycrystal with a crack slab, FP64 fields to the parity tolerances
and mixed-precision macro stress; the crack stays at 1 and the damage next to it follows
the regularised profile from the first increment."""
import dataclasses

import numpy as np
import pytest

from oracle import OracleRVE
from synth import small_polycrystal, make_inputs
from test_gpu_increment import compare

pytestmark = pytest.mark.gpu


def _case():
    # low G_crit and high toughness as in the damage parity case: the source switches on
    # after two increments and the damage grows over several alternating passes
    w = dataclasses.replace(small_polycrystal(n=(12, 8, 6), n_grains=3, seed=5), G_crit=0.004,
                            Gc=100.0, amplitude=0.006)
    inp = make_inputs(w)
    phi0 = np.zeros(w.nvox)
    idx = np.arange(w.nvox).reshape(w.n)
    phi0[idx[4:8, 4, :].ravel()] = 1.0       # a 4 x 1 x 6 crack slab across z
    return w, inp, phi0


def _run(precision, n_inc):
    from paper_2304_01125_amd import RVE
    w, inp, phi0 = _case()
    wp = w.parity()
    gpu = RVE(dict((wp if precision == 0 else w).desc(), pf_dirichlet=1), precision)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], phi0)
    ora = OracleRVE(dict(wp.desc(), pf_dirichlet=1), inp["grain"], inp["quat"], inp["tau_c0"],
                    phi0)
    worst = 0.0
    for k in range(n_inc):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        sg = gpu.step(de, inp["dt"][k])
        so = ora.step(de, inp["dt"][k])
        e = np.abs(np.array(sg["macro_stress"]) - so["macro_stress"]).max() / \
            np.abs(so["macro_stress"]).max()
        worst = max(worst, e)
        print(f"  inc {k}: gpu stag {sg['stag_iters']} pf {sg['pf_iters']} | oracle stag "
              f"{so['stag']} pf {so.get('pf_iters')} | macro stress {e:.2e}", flush=True)
    return gpu, ora, phi0, worst


def test_fp64_increments_match_oracle():
    print("Dirichlet crack 12x8x6, FP64, 4 increments", flush=True)
    gpu, ora, phi0, worst = _run(0, 4)
    assert worst <= 1e-9
    compare(gpu, ora)
    phi = gpu.fields(("damage",))["damage"]
    crack = phi0 >= 1.0
    assert np.all(phi[crack] == 1.0)
    assert phi[~crack].max() > 0.5          # the regularised profile next to the crack
    assert ora.trig.sum() > 100
    gpu.close()


def test_mixed_precision_macro_stress():
    print("Dirichlet crack 12x8x6, mixed precision, 4 increments", flush=True)
    gpu, ora, phi0, worst = _run(1, 4)
    assert worst <= 1e-4
    phi = gpu.fields(("damage",))["damage"]
    assert np.all(phi[phi0 >= 1.0] == 1.0)
    gpu.close()


@pytest.mark.parametrize("free", [0, 1])
def test_degenerate_cracks_match_oracle(free):
    """The crack covers every voxel (nothing to solve: phi stays 1) or all but one."""
    from paper_2304_01125_amd import RVE
    print(f"Dirichlet crack covering all voxels but {free}, 8x8x4", flush=True)
    w = small_polycrystal(n=(8, 8, 4), n_grains=2, seed=3).parity()
    inp = make_inputs(w)
    phi0 = np.ones(w.nvox)
    if free:
        phi0[37] = 0.0
    gpu = RVE(dict(w.desc(), pf_dirichlet=1), 0)
    gpu.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], phi0)
    ora = OracleRVE(dict(w.desc(), pf_dirichlet=1), inp["grain"], inp["quat"], inp["tau_c0"], phi0)
    for k in range(2):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        gpu.step(de, inp["dt"][k])
        ora.step(de, inp["dt"][k])
    phi = gpu.fields(("damage",))["damage"]
    assert np.all(phi[phi0 >= 1.0] == 1.0)
    assert np.abs(phi - ora.phi).max() <= 1e-8
    compare(gpu, ora)
    gpu.close()
