"""Launch one operator building block repeatedly (for profilers and counters).

    python -m paper_2304_01125_amd.passbench --pass x_tangent[,zgrad,...] --n 128 --reps 20 [--mixed]
    python -m paper_2304_01125_amd.passbench --copy-mib 512 --reps 20
    python -m paper_2304_01125_amd.passbench --stream-mib 512 --reps 20

The first form builds a handle on an N^3 grid of the 512-grain Laguerre workload's
material, runs one constitutive update (so the tangent field is populated) and then
enqueues the pass `reps` times (the spectral work buffers hold whatever the arena
held: the timing does not depend on their values); the second times torch's device copy of a buffer of
the given size, the calibration point for hardware byte counters; the third times three
plain torch streams over buffers of the given size (device copy, sum = read only, and
y = x + a z = two reads and one write), the practical HBM ceiling of streaming kernels.
Prints one JSON line with the HIP-event average per launch and the algorithmic bytes.
"""
import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pass", dest="pass_name", default="x_tangent")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--copy-mib", type=float, default=0.0)
    ap.add_argument("--stream-mib", type=float, default=0.0)
    ap.add_argument("--grains", type=int, default=0,
                    help="grains of the microstructure (default N^3/4096; the pass timings do "
                         "not depend on it, its generation time does)")
    a = ap.parse_args()
    import numpy as np
    import torch
    if a.stream_mib > 0:
        n = int(a.stream_mib * 2 ** 20 / 8)
        x = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
        z = torch.empty_like(x).fill_(2.0)
        y = torch.empty_like(x)
        acc = torch.empty((), dtype=torch.float64, device="cuda")
        ops = {"copy": (lambda: y.copy_(x), 2), "sum": (lambda: torch.sum(x, 0, out=acc), 1),
               "triad": (lambda: torch.add(x, z, alpha=0.5, out=y), 3)}
        out = {"bytes_per_operand": 8 * n}
        for name, (f, nops) in ops.items():
            f()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(a.reps):
                f()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1) / a.reps
            out[name] = {"ms": ms, "GB/s": nops * 8 * n / (ms * 1e-3) / 1e9}
        print(json.dumps(out))
        return
    if a.copy_mib > 0:
        n = int(a.copy_mib * 2 ** 20 / 8)
        x = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.reps):
            y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "ms": ms,
                          "GB/s": 16 * n / (ms * 1e-3) / 1e9}))
        return
    from . import RVE, RVE_FP64, RVE_MIXED
    from .rve import PASSES
    from synth import workload, make_inputs
    import dataclasses
    w = dataclasses.replace(workload("laguerre-128-g512"), n=(a.n, a.n, a.n),
                            n_grains=a.grains or max(1, a.n ** 3 // 4096))
    inp = make_inputs(w)
    r = RVE(w.desc(), RVE_MIXED if a.mixed else RVE_FP64)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    r.launch_pass(PASSES["constitutive"], 1)     # populate the tangent field
    for name in a.pass_name.split(","):
        pid = PASSES[name]
        r.launch_pass(pid, 2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(r.stream)
        nbytes = r.launch_pass(pid, a.reps)
        e1.record(r.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        print(json.dumps({"pass": name, "n": a.n, "mixed": a.mixed, "reps": a.reps,
                          "ms": ms, "bytes_per_launch": nbytes,
                          "GB/s": nbytes / (ms * 1e-3) / 1e9}), flush=True)
    r.close()


if __name__ == "__main__":
    main()
