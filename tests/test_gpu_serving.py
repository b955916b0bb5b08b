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


@pytest.mark.parametrize("use_pool", [False, True])
def test_admission_respects_memory_budget(use_pool):
    """Both servers finish every request under a budget that never holds the two largest;
    with use_pool the budget is one library arena (rve_create_in_pool admission), whose
    ranges are all free again at the end."""
    from paper_2304_01125_amd import RVE_MIXED, make_desc, rve_footprint_bytes
    from paper_2304_01125_amd.serve import Server
    gaps, items = _items(4, seed=6)
    sizes = [rve_footprint_bytes(make_desc(w.desc(), RVE_MIXED)) for w, _ in items]
    budget = max(sizes) + min(sizes) - 1          # never two of the largest at once
    srv = Server(RVE_MIXED, max_slots=4, budget_bytes=budget, use_pool=use_pool)
    if use_pool:
        res, wall = srv.run_async(items, np.zeros(len(items)))
        assert all(r["status"] == 0 for r in res), [r["status"] for r in res]
        assert 0 < srv.peak_used <= srv.pool_total <= budget
        assert srv.pool.free_bytes() == (srv.pool_total, srv.pool_total)
    res, wall, ticks = srv.run(items, np.zeros(len(items)))
    assert all(r["status"] == 0 for r in res)
    # the resident footprints never exceeded the budget, and the two largest requests
    # were never resident together
    assert 0 < srv.peak_used <= budget
    big = sorted(range(len(items)), key=lambda i: sizes[i])[-2:]
    assert not any(set(big) <= set(ids) for ids in srv.resident_log)
    assert len(srv.resident_log) == ticks
    srv.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_pool_tick_batches_same_size_solves_bitwise(prec):
    """rve_pool_step runs the CG iterations of same-size handles as shared launches (one
    launch over every handle of the group): four 32^3 polycrystals and a 16^3 one, three
    increments, each bitwise equal to its solve alone; the 32^3 solves did share."""
    import dataclasses
    from paper_2304_01125_amd import RVE
    from paper_2304_01125_amd.rve import rve_pool_step
    from synth import small_polycrystal, make_inputs
    ws = [dataclasses.replace(small_polycrystal(n=32, n_grains=64, seed=s), amplitude=a)
          for s, a in ((1, 0.004), (2, 0.006), (3, 0.008), (4, 0.005))]
    ws.append(small_polycrystal(n=16, n_grains=8, seed=5))
    inps = [make_inputs(w) for w in ws]
    n_inc = 3
    alone = []
    for w, inp in zip(ws, inps):
        r = RVE(w.desc(), prec)
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        for k in range(n_inc):
            r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        alone.append(r.fields(("strain", "stress", "damage", "gs")))
        r.close()
    rs = []
    for w, inp in zip(ws, inps):
        r = RVE(w.desc(), prec)
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        rs.append(r)
    peak = [0.0] * len(rs)
    for k in range(n_inc):
        deps = np.array([[0, inp["deps"][k], 0, 0, 0, 0] for inp in inps])
        dts = np.array([inp["dt"][k] for inp in inps])
        rc, status, stats = rve_pool_step([r.h for r in rs], deps, dts)
        assert rc == 0 and all(s_ == 0 for s_ in status), (rc, status)
        for i, st in enumerate(stats):
            peak[i] = max(peak[i], st["cg_batch"])
    print(f"  largest CG batch per handle: {peak}", flush=True)
    assert max(peak[:4]) >= 2
    for i, r in enumerate(rs):
        f = r.fields(("strain", "stress", "damage", "gs"))
        for key in f:
            assert np.array_equal(f[key], alone[i][key]), (i, key)
        r.close()


def test_pool_admits_by_footprint_and_reuses_released_ranges():
    """rve_create_in_pool: handles take their footprint from the pool's arena until no free
    range fits (RVE_E_NOMEM), a destroyed handle's range is taken again, the pool refuses
    destruction while handles live, and pool handles stepped together with rve_pool_step
    give bitwise the results of a handle in an arena of its own."""
    from paper_2304_01125_amd import (RVE, RvePool, RveError, RVE_MIXED, RVE_E_NOMEM,
                                      RVE_E_STATE, make_desc, rve_footprint_bytes, rve_pool_step)
    from synth import small_polycrystal, make_inputs
    print("pool of 32^3 mixed-precision handles", flush=True)
    w = small_polycrystal(n=(32, 32, 32), n_grains=8, seed=4)
    inp = make_inputs(w)
    fp = (rve_footprint_bytes(make_desc(w.desc(), RVE_MIXED)) + 255) // 256 * 256
    pool = RvePool(5 * fp // 2)
    assert pool.free_bytes()[0] >= 2 * fp
    a = RVE(w.desc(), RVE_MIXED, pool=pool)
    b = RVE(w.desc(), RVE_MIXED, pool=pool)
    with pytest.raises(RveError) as e:
        RVE(w.desc(), RVE_MIXED, pool=pool)
    assert e.value.code == RVE_E_NOMEM
    with pytest.raises(RveError) as e:
        pool.close()
    assert e.value.code == RVE_E_STATE
    a.close()
    c = RVE(w.desc(), RVE_MIXED, pool=pool)        # the released range is taken again
    ref = RVE(w.desc(), RVE_MIXED)
    for r in (b, c, ref):
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(3):
        de = [0, inp["deps"][k], 0, 0, 0, 0]
        rc, status, _ = rve_pool_step([b.h, c.h], [de, de], [inp["dt"][k]] * 2)
        assert rc == 0 and status == [0, 0]
        ref.step(de, inp["dt"][k])
    fr = ref.fields(("strain", "stress"))
    for r in (b, c):
        f = r.fields(("strain", "stress"))
        for name in ("strain", "stress"):
            assert np.array_equal(f[name], fr[name]), name
    for r in (b, c, ref):
        r.close()
    tot, largest = pool.free_bytes()
    assert tot == largest and tot >= 2 * fp          # the free ranges merged again
    pool.close()


def test_pool_first_fit_with_mixed_sizes():
    """Handles of three sizes in one pool: the free bytes drop by each handle's footprint
    rounded up to 256 B, a small handle takes the gap a larger one left (first fit, lowest
    offset), releases that are not adjacent stay separate ranges, and the last release
    merges everything back into one range.  The handle in the gap then solves an increment
    bitwise like a handle in its own arena."""
    from paper_2304_01125_amd import RVE, RvePool, RVE_FP64, make_desc, rve_footprint_bytes
    from synth import small_polycrystal, make_inputs
    print("pool with 8^3, 16^3 and 24^3 handles", flush=True)
    ws = {n: small_polycrystal(n=(n, n, n), n_grains=4, seed=n) for n in (8, 16, 24)}
    fp = {n: (rve_footprint_bytes(make_desc(w.desc(), RVE_FP64)) + 255) // 256 * 256
          for n, w in ws.items()}
    assert fp[8] < fp[16] < fp[24]
    pool = RvePool(fp[16] + fp[24] + fp[16] + 4096)
    total = pool.free_bytes()[0]
    a = RVE(ws[16].desc(), RVE_FP64, pool=pool)         # [a | b | c | rest]
    b = RVE(ws[24].desc(), RVE_FP64, pool=pool)
    c = RVE(ws[16].desc(), RVE_FP64, pool=pool)
    used = fp[16] + fp[24] + fp[16]
    assert pool.free_bytes() == (total - used, total - used)
    b.close()                                          # gap of fp[24] between a and c
    assert pool.free_bytes() == (total - used + fp[24], fp[24])
    d = RVE(ws[8].desc(), RVE_FP64, pool=pool)          # first fit: into the gap
    assert pool.free_bytes() == (total - used + fp[24] - fp[8], fp[24] - fp[8])
    inp = make_inputs(ws[8])
    ref = RVE(ws[8].desc(), RVE_FP64)
    for r in (d, ref):
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        r.step([0, inp["deps"][0], 0, 0, 0, 0], inp["dt"][0])
    fd, fr = d.fields(("strain", "stress")), ref.fields(("strain", "stress"))
    for k in ("strain", "stress"):
        assert np.array_equal(fd[k], fr[k]), k
    ref.close()
    a.close()                                          # [free | d | gap | c | rest]
    tot, largest = pool.free_bytes()
    assert tot == total - fp[16] - fp[8] and largest == max(fp[16], fp[24] - fp[8], total - used)
    c.close()
    d.close()
    assert pool.free_bytes() == (total, total)
    pool.close()
