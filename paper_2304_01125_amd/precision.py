"""Mixed precision against FP64 on one workload: per-increment macro stress error and
per-field relative L2 errors of the FP32-bulk run against the FP64 run (both on the GPU;
the FP64 path itself matches the CPU oracle to ~1e-15 on the parity workloads).

    python -m paper_2304_01125_amd.precision --workload voronoi-256-g4096-hard --incs 3
"""
import argparse
import json
import time

import numpy as np


def compare(name, incs):
    import torch
    from . import RVE, RVE_FP64, RVE_MIXED
    from synth import workload, make_inputs
    w = workload(name)
    inp = make_inputs(w)
    out = {"workload": name, "increments": incs}
    runs = {}
    for prec, label in ((RVE_FP64, "fp64"), (RVE_MIXED, "mixed")):
        r = RVE(w.desc(), prec)
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        macro, kry = [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(incs):
            st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
            macro.append(st["macro_stress"])
            kry += st["krylov_iters"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        runs[label] = dict(macro=np.array(macro), fields=r.fields(("strain", "stress", "eps_p",
                                                                    "gs", "wp", "damage")))
        out[label] = {"voxel_iters_per_s": round(w.nvox * kry / dt, 1),
                      "ms_per_increment": round(1e3 * dt / incs, 1), "krylov_iters": kry}
        r.close()
        del r
    a, b = runs["mixed"], runs["fp64"]
    out["macro_stress_rel_err"] = [float(v) for v in np.abs(a["macro"] - b["macro"]).max(1) /
                                   np.abs(b["macro"]).max(1)]
    out["field_rel_l2"] = {k: float(np.linalg.norm(a["fields"][k] - b["fields"][k]) /
                                    max(np.linalg.norm(b["fields"][k]), 1e-300))
                           for k in a["fields"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="voronoi-256-g4096-hard")
    ap.add_argument("--incs", type=int, default=3)
    a = ap.parse_args()
    print(json.dumps(compare(a.workload, a.incs)), flush=True)


if __name__ == "__main__":
    main()
