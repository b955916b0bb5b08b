"""Continuous-batching server: concurrent solves give the same results as solving each
request alone (bitwise: every reduction has a fixed order and the solves share nothing),
admission respects the memory budget, and every request completes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _items(n_req=6, seed=5):
    from synth import serving_requests
    from paper_2304_01125_amd.serve import prepare
    factor, gaps, reqs = serving_requests(n_req, seed, grids=(16, 24, 32))
    return gaps, prepare(reqs)


@pytest.mark.parametrize("slots", [3])
def test_each_result_alone_equals_result_in_the_mix(slots):
    from paper_2304_01125_amd import RVE_MIXED
    from paper_2304_01125_amd.serve import Server, run_serial
    gaps, items = _items()
    alone, _ = run_serial(items, RVE_MIXED, keep_fields=True)
    arrivals = np.cumsum(gaps) * 0.01            # dense arrivals: several solves overlap
    srv = Server(RVE_MIXED, max_slots=slots)
    mixed, wall, ticks = srv.run(items, arrivals, keep_fields=True)
    print(f"  {len(items)} requests, {ticks} ticks, wall {wall:.2f} s", flush=True)
    assert ticks < sum(len(inp["deps"]) for _, inp in items)      # solves did overlap
    for a, b in zip(alone, mixed):
        assert b["status"] == 0
        for k in ("strain", "stress", "damage"):
            assert np.array_equal(a["fields"][k], b["fields"][k]), (a["id"], k)
    # slot-per-thread server: same results, solves overlap on their own streams
    res, wall = srv.run_async(items, arrivals, keep_fields=True)
    for a, b in zip(alone, res):
        assert b["status"] == 0
        for k in ("strain", "stress", "damage"):
            assert np.array_equal(a["fields"][k], b["fields"][k]), (a["id"], k)


def test_admission_respects_memory_budget():
    from paper_2304_01125_amd import RVE_MIXED, make_desc, rve_footprint_bytes
    from paper_2304_01125_amd.serve import Server
    gaps, items = _items(4, seed=6)
    sizes = [rve_footprint_bytes(make_desc(w.desc(), RVE_MIXED)) for w, _ in items]
    budget = max(sizes) + min(sizes) - 1          # never two of the largest at once
    srv = Server(RVE_MIXED, max_slots=4, budget_bytes=budget)
    res, wall, ticks = srv.run(items, np.zeros(len(items)))
    assert all(r["status"] == 0 for r in res)
    # the resident footprints never exceeded the budget, and the two largest requests
    # were never resident together
    assert 0 < srv.peak_used <= budget
    big = sorted(range(len(items)), key=lambda i: sizes[i])[-2:]
    assert not any(set(big) <= set(ids) for ids in srv.resident_log)
    assert len(srv.resident_log) == ticks
