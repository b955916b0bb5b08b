"""Live timing of the row tangent pass inside the solver's CG iterations (the benchmark's
roofline measurement): one timed launch per CG iteration that ran (the no-op launches after
convergence are not counted), or per every-th iteration of each solve, positive durations,
and results bitwise equal to an untimed run (the timed iterations are launched eagerly
instead of replayed from graphs)."""
import numpy as np
import pytest

from synth import small_polycrystal, make_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [(32, 32, 32), (12, 8, 6)])
def test_live_timing_counts_every_cg_iteration(n):
    from paper_2304_01125_amd import RVE
    w = small_polycrystal(n=n, n_grains=8, seed=3)
    inp = make_inputs(w)
    out = []
    for every in (0, 1, 8):
        r = RVE(w.desc())
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        if every:
            r.time_pass("x_tangent", True, every=every)
        kry = newton = 0
        for k in range(3):
            st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
            kry += st["krylov_iters"]
            newton += st["newton_iters"]
        launches, ms = r.pass_time()
        print(f"  {n} every {every}: krylov {kry} in {newton} solves, timed launches "
              f"{launches}, {ms:.3f} ms", flush=True)
        if every == 1:
            assert launches == kry and ms > 0.0
        elif every:
            # iterations 0, 8, 16, ... of each CG solve (one solve per Newton iteration)
            assert kry / every <= launches <= kry / every + newton and ms > 0.0
        else:
            assert launches == 0 and ms == 0.0
        out.append(r.fields(("strain", "stress")))
        r.close()
    for name in out[0]:
        assert np.array_equal(out[0][name], out[1][name]), name
        assert np.array_equal(out[0][name], out[2][name]), name
