"""Continuous-batching server of independent RVE solves on one GPU.

Requests (a microstructure, a grid size and a load history each) arrive over time.
The server keeps up to `max_slots` solves resident in HBM, admits a waiting request as
soon as a slot is free and its arena footprint fits the memory budget, and advances
all resident solves by one load increment per tick with ``rve_pool_step`` (one HIP
stream per slot, so their kernels overlap on the device).  With ``use_pool`` the budget is
one device arena held by the library (``rve_pool_create``): a request is admitted when
``rve_create_in_pool`` finds a free range for its footprint, and its range returns to the
pool when its handle is destroyed.  A request that finishes its
last increment releases its slot and memory at once; newcomers join at the next tick,
without waiting for the others to finish.  Reported: solves/s, p50/p99 latency
(arrival to completion) and the same for serial solves.

    python -m paper_2304_01125_amd.serve --requests 400 [--slots 8] [--mode async|tick|both]
        [--pool] [--budget-gib 32] [--capacity SOLVES_PER_S] [--low-rate 0.5] [--json out.json]
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def prepare(reqs, workers=None):
    """Client-side inputs of every request (microstructure and load history)."""
    from synth import request_workload, make_inputs
    items = []
    if workers and workers > 1:
        # spawned (not forked) workers: the caller may already have initialised the GPU,
        # and a forked copy of a HIP-initialised process is not safe to run
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        ctx = multiprocessing.get_context("spawn")
        with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
            inps = list(ex.map(_make, reqs))
    else:
        inps = [_make(r) for r in reqs]
    for r, inp in zip(reqs, inps):
        items.append((request_workload(r), inp))
    return items


def _make(req):
    from synth import request_workload, make_inputs
    return make_inputs(request_workload(req))


class Server:
    def __init__(self, precision, max_slots=8, budget_bytes=32 << 30, device=0, use_pool=False):
        import torch
        from . import load, RvePool
        load()
        self.torch = torch
        self.precision = precision
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(max_slots)]
        self.pool = RvePool(budget_bytes, device) if use_pool else None
        self.pool_total = self.pool.free_bytes()[0] if use_pool else 0
        self.peak_used = 0                # largest resident footprint sum (bytes)

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool = None

    def _admit(self, w, slot):
        """A handle for workload w on the slot's stream, or None when the pool has no free
        range for it yet; raises RveError(RVE_E_NOMEM) for a request larger than the whole
        pool, which no release can admit."""
        from .rve import RVE, RveError, RVE_E_NOMEM
        if self.pool is None:
            return RVE(w.desc(), self.precision, stream=self.streams[slot])
        try:
            r = RVE(w.desc(), self.precision, stream=self.streams[slot], pool=self.pool)
            # resident bytes from the pool itself: a handle returns its range at close(),
            # before the server's own count of resident bytes drops
            self.peak_used = max(self.peak_used, self.pool_total - self.pool.free_bytes()[0])
            return r
        except RveError as e:
            if e.code == RVE_E_NOMEM and self.pool.free_bytes()[0] < self.pool_total:
                return None
            raise

    def run(self, items, arrivals, keep_fields=False, log=None):
        """items: [(workload, inputs)], arrivals: seconds after start (non-decreasing).
        Returns per-request dicts (latency, status, ...) and the wall time."""
        from .rve import RveError, rve_pool_step
        from . import make_desc, rve_footprint_bytes
        torch = self.torch
        n = len(items)
        order = list(np.argsort(arrivals, kind="stable"))
        out = [None] * n
        waiting, active = [], []          # active: dicts with slot, handle, k
        free_slots = list(range(self.max_slots))
        used = 0
        self.peak_used = 0                # largest resident footprint sum (bytes)
        self.resident_log = []            # request ids resident at each tick
        t0 = time.perf_counter()
        nxt = 0
        ticks = 0
        while nxt < n or waiting or active:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[order[nxt]] <= now:
                waiting.append(order[nxt])
                nxt += 1
            # admission: free slot and memory
            while waiting and free_slots:
                i = waiting[0]
                w, inp = items[i]
                need = rve_footprint_bytes(make_desc(w.desc(), self.precision))
                if self.pool is None and used + need > self.budget and active:
                    break
                slot = free_slots[0]
                try:
                    r = self._admit(w, slot)
                except RveError as e:           # larger than the whole pool
                    waiting.pop(0)
                    out[i] = dict(id=i, n=w.n[0], status=e.code, latency=now - arrivals[i],
                                  queued=0.0, krylov_iters=0, macro_stress=None, error=str(e))
                    continue
                if r is None:
                    break
                waiting.pop(0)
                free_slots.pop(0)
                r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
                used += r.footprint
                if self.pool is None:
                    self.peak_used = max(self.peak_used, used)
                active.append(dict(i=i, slot=slot, rve=r, k=0, t_admit=now, iters=0))
            if not active:
                if nxt < n:
                    time.sleep(max(0.0, min(0.01, arrivals[order[nxt]] - now)))
                continue
            deps = np.zeros((len(active), 6))
            dts = np.zeros(len(active))
            for a_i, a in enumerate(active):
                w, inp = items[a["i"]]
                deps[a_i, 1] = inp["deps"][a["k"]]
                dts[a_i] = inp["dt"][a["k"]]
            self.resident_log.append([a["i"] for a in active])
            rc, status, stats = rve_pool_step([a["rve"].h for a in active], deps, dts)
            ticks += 1
            done_now = time.perf_counter() - t0
            still = []
            for a, s, st in zip(active, status, stats):
                a["k"] += 1
                a["iters"] += st["krylov_iters"]
                w, inp = items[a["i"]]
                if s != 0 or a["k"] == len(inp["deps"]):
                    rec = dict(id=a["i"], n=w.n[0], status=s, latency=done_now - arrivals[a["i"]],
                               queued=a["t_admit"] - arrivals[a["i"]], krylov_iters=a["iters"],
                               macro_stress=st["macro_stress"])
                    if keep_fields:
                        rec["fields"] = a["rve"].fields(("strain", "stress", "damage"))
                    out[a["i"]] = rec
                    used -= a["rve"].footprint
                    a["rve"].close()
                    free_slots.append(a["slot"])
                    if log:
                        log(f"request {a['i']} ({w.n[0]}^3) done: status {s}, "
                            f"latency {rec['latency']:.3f} s")
                else:
                    still.append(a)
            active = still
        wall = time.perf_counter() - t0
        return out, wall, ticks


    def run_async(self, items, arrivals, keep_fields=False, log=None):
        """Slot-per-thread variant: each slot's host thread takes the oldest arrived
        request that fits the memory budget, runs its increments on the slot's stream,
        releases its memory and takes the next one; slots never wait for each other."""
        import threading
        n = len(items)
        order = list(np.argsort(arrivals, kind="stable"))
        out = [None] * n
        lock = threading.Lock()
        state = {"next": 0, "used": 0}
        self.peak_used = 0
        from . import make_desc, rve_footprint_bytes
        need = [rve_footprint_bytes(make_desc(w.desc(), self.precision)) for w, _ in items]
        t0 = time.perf_counter()

        def worker(slot):
            torch = self.torch
            torch.cuda.set_device(self.device)
            while True:
                with lock:
                    if state["next"] >= n:
                        return
                    i = order[state["next"]]
                    wait = arrivals[i] - (time.perf_counter() - t0)
                    r = err = None
                    if wait > 0 or (self.pool is None and state["used"] + need[i] > self.budget):
                        i = None
                    else:
                        if self.pool is not None:
                            # created under the lock, so requests take pool ranges in
                            # arrival order
                            try:
                                r = self._admit(items[i][0], slot)
                            except Exception as e:
                                err = e
                            if r is None and err is None:
                                i = None
                        if i is not None:
                            state["next"] += 1
                            state["used"] += need[i]
                            if self.pool is None:
                                self.peak_used = max(self.peak_used, state["used"])
                if i is None:
                    time.sleep(0.002)
                    continue
                w, inp = items[i]
                t_admit = time.perf_counter() - t0
                rec = dict(id=i, n=w.n[0], status=None, latency=None,
                           queued=t_admit - arrivals[i], krylov_iters=0, macro_stress=None)
                try:
                    if err is not None:
                        raise err
                    if r is None:
                        r = self._admit(w, slot)
                    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
                    it, st = 0, {"status": 0, "macro_stress": None}
                    for k in range(len(inp["deps"])):
                        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], check=False)
                        it += st["krylov_iters"]
                        if st["status"] != 0:
                            break
                    rec.update(status=st["status"], krylov_iters=it, macro_stress=st["macro_stress"])
                    if keep_fields:
                        rec["fields"] = r.fields(("strain", "stress", "damage"))
                except Exception as e:               # a failed request must not hold its memory
                    rec.update(status=-1000, error=str(e))
                finally:
                    if r is not None:
                        r.close()
                        del r
                    rec["latency"] = time.perf_counter() - t0 - arrivals[i]
                    out[i] = rec
                    with lock:
                        state["used"] -= need[i]
                if log:
                    log(f"request {i} ({w.n[0]}^3) done on slot {slot}: status {rec['status']}, "
                        f"latency {rec['latency']:.3f} s")

        threads = [threading.Thread(target=worker, args=(s_,)) for s_ in range(self.max_slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        return out, time.perf_counter() - t0


def run_serial(items, precision, keep_fields=False, log=None):
    """Each request alone, back to back (no queueing): per-request solve times."""
    import torch
    from .rve import RVE
    out = []
    t0 = time.perf_counter()
    for i, (w, inp) in enumerate(items):
        t1 = time.perf_counter()
        r = RVE(w.desc(), precision)
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        it = 0
        for k in range(len(inp["deps"])):
            st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], check=False)
            it += st["krylov_iters"]
            if st["status"] != 0:
                break
        torch.cuda.synchronize()
        rec = dict(id=i, n=w.n[0], status=st["status"], latency=time.perf_counter() - t1,
                   krylov_iters=it, macro_stress=st["macro_stress"])
        if keep_fields:
            rec["fields"] = r.fields(("strain", "stress", "damage"))
        out.append(rec)
        r.close()
        if log:
            log(f"serial request {i} ({w.n[0]}^3): status {rec['status']}, "
                f"{1e3 * rec['latency']:.1f} ms")
    return out, time.perf_counter() - t0


def summary(recs, wall):
    lat = np.array([r["latency"] for r in recs])
    return {"solves_per_s": round(len(recs) / wall, 3), "p50_ms": round(1e3 * np.percentile(lat, 50), 1),
            "p99_ms": round(1e3 * np.percentile(lat, 99), 1), "n": len(recs),
            "wall_s": round(wall, 2)}


def serve_benchmark(n_req=400, slots=8, seed=4, workers=8, log=None, items=None, low_rate=0.5,
                    modes=("async", "tick"), use_pool=False, capacity=None, budget_bytes=32 << 30):
    """Serial plain-FP64 baseline, then the mixed-precision server in each of `modes` on the
    Poisson stream at rate factor x the serial capacity, and at `low_rate` x its own measured
    throughput (latency without a growing queue).  Mode "async": each slot runs its request's
    increments back to back on its own stream and host thread; "tick": one rve_pool_step per
    tick, the CG iterations of same-size requests in shared launches.  The first mode fills
    `server_mixed` and `server_mixed_below_capacity`, every mode `<mode>`.  Returns a
    JSON-able dict.  `items`: the prepared requests (else prepared here); `use_pool`: admission
    by first fit in one library-held arena (rve_create_in_pool) instead of the budget sum;
    `capacity`: the serial solves/s that sets the arrival rate, given instead of measured
    (the serial run is skipped); low_rate <= 0 skips the below-capacity runs."""
    from synth import serving_requests
    from . import RVE_FP64, RVE_MIXED
    factor, gaps, reqs = serving_requests(n_req, seed)
    if items is None:
        items = prepare(reqs, workers)
    if log:
        log(f"prepared {len(items)} requests")
    if capacity is None:
        serial, wall_s = run_serial(items, RVE_FP64, log=log)
        cap = len(serial) / wall_s
    else:
        serial, cap = None, float(capacity)
    lam = factor * cap
    arrivals = np.cumsum(gaps) / lam
    srv = Server(RVE_MIXED, max_slots=slots, budget_bytes=budget_bytes, use_pool=use_pool)
    out = {"requests": n_req, "slots": slots, "rate_factor": round(factor, 3),
           "arrival_rate_per_s": round(lam, 3),
           "admission": "pool (first fit)" if use_pool else "budget sum",
           "budget_gib": round(budget_bytes / 2 ** 30, 3)}
    if serial is not None:
        out["completed_serial"] = sum(1 for r in serial if r["status"] == 0)
        out["serial_fp64"] = summary(serial, wall_s)
    else:
        out["serial_capacity_given"] = cap
    for i, mode in enumerate(modes):
        def serve(arr):
            if mode == "async":
                res, wall = srv.run_async(items, arr, log=log)
                return res, wall, None
            return srv.run(items, arr, log=log)

        res, wall, ticks = serve(arrivals)
        m = {"completed": sum(1 for r in res if r["status"] == 0),
             "server_mixed": summary(res, wall),
             "peak_resident_gib": round(srv.peak_used / 2 ** 30, 3)}
        if ticks is not None:
            m["ticks"] = ticks
        # below capacity: arrivals at low_rate x this server's throughput under the stream
        if low_rate > 0:
            lam_low = low_rate * len(res) / wall
            res2, wall2, _ = serve(np.cumsum(gaps) / lam_low)
            m["server_mixed_below_capacity"] = dict(summary(res2, wall2),
                                                   arrival_rate_per_s=round(lam_low, 3))
        out[mode] = m
        if i == 0:
            out["mode"] = mode
            out["completed"] = m["completed"]
            out["server_mixed"] = m["server_mixed"]
            if low_rate > 0:
                out["server_mixed_below_capacity"] = m["server_mixed_below_capacity"]
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--json", default=None)
    ap.add_argument("--mode", choices=["tick", "async", "both"], default="both")
    ap.add_argument("--pool", action="store_true",
                    help="admit by first fit in one library-held arena (rve_create_in_pool)")
    ap.add_argument("--budget-gib", type=float, default=32.0)
    ap.add_argument("--capacity", type=float, default=None,
                    help="serial solves/s that sets the arrival rate (skips the serial run)")
    ap.add_argument("--low-rate", type=float, default=0.5,
                    help="below-capacity arrival rate / server throughput (0: skip)")
    a = ap.parse_args()
    modes = ("async", "tick") if a.mode == "both" else (a.mode,)
    res = serve_benchmark(a.requests, a.slots, a.seed, a.workers,
                          log=lambda m: print(m, file=sys.stderr, flush=True), modes=modes,
                          use_pool=a.pool, capacity=a.capacity, low_rate=a.low_rate,
                          budget_bytes=int(a.budget_gib * 2 ** 30))
    print(json.dumps(res), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
