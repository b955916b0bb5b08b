"""The request stream of the serving workload: independent solves of different grids.

Each request: grid N^3 with N uniform in {32, 48, 64, 96}, a periodic Voronoi
microstructure with N^3/512 grains from its own seed, uniform random orientations,
strain amplitude uniform in [0.3 %, 0.8 %], strain ratio R in {-1, 0}, one cycle of 20
increments.  Arrivals form a Poisson process; its rate is a factor drawn uniformly in
[1, 4] times a capacity the caller measures (the serial plain-FP64 throughput), so the
stream carries unit-rate exponential gaps that the caller scales.
"""
import numpy as np

from .workloads import Workload

GRIDS = (32, 48, 64, 96)


def serving_requests(n_req=400, seed=4, grids=GRIDS):
    """Returns (rate_factor, unit_gaps[n_req], requests[n_req] as dicts)."""
    rng = np.random.default_rng(seed)
    factor = float(rng.uniform(1.0, 4.0))
    reqs = []
    for i in range(n_req):
        n = int(grids[rng.integers(len(grids))])
        reqs.append(dict(id=i, n=n, amplitude=float(rng.uniform(0.003, 0.008)),
                         ratio=int((-1, 0)[rng.integers(2)]), seed=int(rng.integers(2 ** 31 - 1))))
    gaps = rng.exponential(1.0, n_req)
    return factor, gaps, reqs


def request_workload(req, **kw):
    n = req["n"]
    return Workload(name=f"request-{req['id']}-{n}", n=(n, n, n), n_grains=max(1, n ** 3 // 512),
                    seed=req["seed"], amplitude=req["amplitude"], ratio=req["ratio"], cycles=1,
                    incs_per_cycle=20, **kw)
