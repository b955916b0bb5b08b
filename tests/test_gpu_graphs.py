"""CG iterations replayed as HIP graphs give bitwise the same increments as the same
launches made one by one.  Every increment replays the two captured graphs (one per
iteration parity) many times, with eager launches, host reads and synchronisations of
the Newton and staggered loops between the replays; all of them are compared."""
import os

import numpy as np
import pytest

from synth import small_polycrystal, workload, make_inputs

pytestmark = pytest.mark.gpu


def _run(w, precision, graphs, n_inc, mask=0):
    from paper_2304_01125_amd import RVE
    old = os.environ.get("RVE_GRAPHS")
    os.environ["RVE_GRAPHS"] = "1" if graphs else "0"
    try:
        inp = make_inputs(w)
        r = RVE(w.desc(), precision)
    finally:
        if old is None:
            del os.environ["RVE_GRAPHS"]
        else:
            os.environ["RVE_GRAPHS"] = old
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    out = []
    for k in range(n_inc):
        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], dsig6=np.zeros(6),
                    stress_mask=mask)
        out.append((st["krylov_iters"], r.fields(("strain", "stress", "damage", "gs"))))
    r.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("grid", ["fused", "unfused"])
def test_graph_replays_equal_eager_launches(precision, grid):
    if grid == "fused":          # 32^3: register DFTs and the fused z passes
        w = small_polycrystal(n=(32, 32, 32), n_grains=8, seed=3)
    else:                        # 12 x 8 x 6: runtime-length FFTs, unfused operator
        w = small_polycrystal(n=(12, 8, 6), n_grains=4, seed=7)
    a = _run(w, precision, True, 3)
    b = _run(w, precision, False, 3)
    for k, ((ka, fa), (kb, fb)) in enumerate(zip(a, b)):
        print(f"  inc {k}: krylov graphs {ka} eager {kb}", flush=True)
        assert ka == kb
        for name in fa:
            assert np.array_equal(fa[name], fb[name]), (k, name)


@pytest.mark.parametrize("grid", ["fused", "unfused"])
def test_graph_replays_equal_eager_launches_under_stress_control(grid):
    # uniaxial stress: the graphs hold the macro strain / stress launches as well
    if grid == "fused":
        w = small_polycrystal(n=(32, 32, 32), n_grains=8, seed=3)
    else:
        w = small_polycrystal(n=(12, 8, 6), n_grains=4, seed=7)
    a = _run(w, 0, True, 3, mask=0b111101)
    b = _run(w, 0, False, 3, mask=0b111101)
    for k, ((ka, fa), (kb, fb)) in enumerate(zip(a, b)):
        print(f"  inc {k}: krylov graphs {ka} eager {kb}", flush=True)
        assert ka == kb
        for name in fa:
            assert np.array_equal(fa[name], fb[name]), (k, name)

