"""The allocation-free entry point rve_create_noalloc (the library's static device arena
in place of a caller-allocated one) against rve_create with a caller arena: the same
increments through the C ABI give identical fields, on two handles in a row (the second
on a smaller grid, in the array the first one left behind); a second handle while one is
alive is refused."""
import numpy as np
import pytest

from synth import small_polycrystal, make_inputs

pytestmark = pytest.mark.gpu


def _run(w, noalloc, n_inc=3):
    from paper_2304_01125_amd import RVE
    inp = make_inputs(w)
    r = RVE(w.desc(), noalloc=noalloc)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    stats = []
    for k in range(n_inc):
        stats.append(r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k]))
    f = r.fields(("strain", "stress", "damage", "gs", "wp", "eps_p", "rho_ssd", "rho_gnd"))
    return r, f, stats


@pytest.mark.parametrize("n", [(16, 16, 16), (12, 8, 6)])
def test_noalloc_handle_matches_arena_handle(n):
    print(f"noalloc {n}", flush=True)
    w = small_polycrystal(n=n, n_grains=4, seed=7).parity()
    ref, f_ref, st_ref = _run(w, noalloc=False)
    ref.close()
    r, f, st = _run(w, noalloc=True)
    r.close()
    for a, b in zip(st_ref, st):
        assert a["krylov_iters"] == b["krylov_iters"] and a["newton_iters"] == b["newton_iters"]
    for k in f_ref:
        print(f"  {k}: max |diff| {np.abs(f[k] - f_ref[k]).max():.2e}", flush=True)
        assert np.array_equal(f[k], f_ref[k]), k


def test_second_noalloc_handle_is_refused_while_one_is_alive():
    from paper_2304_01125_amd import RVE, RveError, RVE_E_STATE
    w = small_polycrystal(n=(8, 8, 8), n_grains=2, seed=1)
    a = RVE(w.desc(), noalloc=True)
    with pytest.raises(RveError) as e:
        RVE(w.desc(), noalloc=True)
    assert e.value.code == RVE_E_STATE
    a.close()
    b = RVE(w.desc(), noalloc=True)          # released by the first handle's close
    b.close()
