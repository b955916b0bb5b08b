#!/usr/bin/env python3
"""Benchmark: voxel-iterations per second of the FFT crystal-plasticity phase-field
increment on one GPU.

A step is one load increment (Algorithm 1: constitutive updates, Newton-Krylov
momentum solve with the Green-operator preconditioner, phase-field solve, history
commit, GND update) of the 128^3 polycrystal with 512 log-normal Laguerre grains,
fully reversed strain cycling at +-0.5 %, at the paper's production tolerances.
A voxel-iteration is one application of the momentum operator to one voxel; the
rate counts every operator application of the timed increments over their whole
wall time (constitutive work, phase field, commit and host synchronisation
included).  Inputs are resident on the GPU before timing starts.

Printed: one JSON line with the FP64 rate, the mixed-precision rate and its macro
stress error against the FP64 run, the roofline of the dominant operator kernel
(HIP events on the library's stream around each of its launches inside the timed
increments; the other passes timed in isolation), the FP64 rate of the same increments with the
paper's GMRES(30) in place of CG, with the rotated-scheme discrete derivative and under uniaxial stress (mixed macroscopic control),
a short serving run (a 40-request seeded stream of 32^3-96^3 solves: mixed-precision
server against serial FP64 solves, solves/s and p50/p99 latency), the FP64 rate of the same grid with the
paper's thermally activated flow rule and Table 1 material in yielding increments (also
with the GND-coupled Taylor strength), the headline increments with finite-strain
kinematics, a 256 x 256 x 1 plate in pointwise plane stress, and the CPU oracle timed on a
bounded sample.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iters/s at 128³ (FP64 vs mixed, stated error); served solves/s + p99"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="laguerre-128-g512")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-material", action="store_true",
                    help="skip the thermally-activated-flow leg (Table 1 material)")
    ap.add_argument("--no-stress-control", action="store_true",
                    help="skip the uniaxial-stress (mixed control) leg")
    ap.add_argument("--no-rotated", action="store_true",
                    help="skip the rotated-scheme (discrete derivative) leg")
    ap.add_argument("--gmres-restart", type=int, default=10,
                    help="restart length m of the GMRES leg (the paper does not fix it; 10 "
                         "measured fastest of 10, 20 and 30 at 128^3)")
    ap.add_argument("--no-gmres", action="store_true",
                    help="skip the GMRES(m) leg (the paper's Krylov solver)")
    ap.add_argument("--deriv", choices=["spectral", "rotated"], default="spectral",
                    help="derivative of the FP64 and mixed legs")
    ap.add_argument("--serve-slots", type=int, default=16,
                    help="resident solves of the serving leg's server (80 requests arriving at "
                         "once: 5.3 solves/s with 16, 4.8 with 8)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="requests of the serving leg (0: skip); the committed serving "
                         "summary uses 400")
    ap.add_argument("--pass-reps", type=int, default=20)
    ap.add_argument("--no-damage", action="store_true",
                    help="skip the damage leg (phase field active in the timed increments)")
    ap.add_argument("--no-finite", action="store_true",
                    help="skip the finite-strain leg (headline grid and load, GMRES(30))")
    ap.add_argument("--no-gnd", action="store_true",
                    help="skip the GND-coupled hardening leg (Table 1 material)")
    ap.add_argument("--no-plate", action="store_true",
                    help="skip the plane-stress plate leg (256 x 256 x 1)")
    ap.add_argument("--damage-gcrit-pow", type=int, default=10,
                    help="the damage leg's G_crit = 4 J/m^2 / 2^k")
    ap.add_argument("--damage-gc", type=float, default=100.0,
                    help="the damage leg's fracture toughness G_c in J/m^2 (growth stays "
                         "stable over the timed increments at 100; at 20 it is not)")
    return ap.parse_args()


LIVE_EVERY = 8     # CG iterations per live-timed launch of the roofline kernel


def run_leg(RVE, precision, desc, inp, warmup, steps, torch, stress_mask=0, live=False):
    r = RVE(desc, precision)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    macro = []
    kw = dict(dsig6=np.zeros(6), stress_mask=stress_mask) if stress_mask else {}
    for k in range(warmup):
        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], **kw)
        macro.append(st["macro_stress"])
    if live:            # HIP events around the row tangent pass of every 8th CG iteration of
        # the timed increments (a recording launch costs the kernels next to it a few us)
        r.time_pass("x_tangent", True, every=LIVE_EVERY)
        r.pass_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kry = 0
    stats = []
    for k in range(warmup, warmup + steps):
        st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], **kw)
        kry += st["krylov_iters"]
        stats.append(st)
        macro.append(st["macro_stress"])
        print(f"# step {k}: {st['ms_total']:.1f} ms, newton {st['newton_iters']}, "
              f"krylov {st['krylov_iters']}, stag {st['stag_iters']}, pf {st['pf_iters']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if live:
        r.live = r.pass_time()
        r.time_pass("x_tangent", False)
    return r, dt, kry, stats, np.array(macro)


def time_passes(r, torch, reps):
    """Average duration of each operator building block, HIP events on the library's
    stream, and its algorithmic HBM bytes per launch."""
    from paper_2304_01125_amd.rve import PASSES
    from paper_2304_01125_amd import RveError
    out = {}
    s = r.stream
    for name in ("fft_z", "fft_y", "x_tangent", "grad", "div", "zgrad", "zdiv", "precond",
                 "matvec"):
        pid = PASSES[name]
        try:
            r.launch_pass(pid, 2)                   # warm
        except RveError:                            # no fused z pass on this grid
            continue
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        nbytes = r.launch_pass(pid, reps)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "bytes": nbytes, "gbs": nbytes / (ms * 1e-3) / 1e9}
    return out


def measured_traffic(kernel, n):
    """HBM bytes per launch of `kernel` (FP64, n^3) from the committed rocprofv3 counter
    summary profiles/<kernel>_fp64_<n>_traffic.md, or None when there is none or the
    kernel source has changed since the counters were taken (the summary records the
    SHA-256 of the source file that holds the kernel)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_fp64_{n}_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    src = re.search(r"(?i)source: `([^`]+)` sha256 `([0-9a-f]{64})`", txt)
    val = re.search(r"measured traffic per launch: ([0-9.]+) MB", txt)
    if not src or not val:
        return None
    with open(os.path.join(ROOT, src.group(1)), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != src.group(2):
            return None
    return float(val.group(1)) * 1e6


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, inp, gpu_stats, first, n_apply=6, stride=64):
    """The CPU oracle on a bounded sample of the same workload, scaled to voxel-iters/s.

    Sample: (a) n_apply applications of the oracle's preconditioned momentum operator on
    the full grid with the elastic tangent of the microstructure; (b) the oracle's return
    map and (c) its phase-field source (trial plastic work and the spectral tensile energy)
    on every stride-th voxel at the macroscopic strain of the first timed increment
    (increment index ``first``), scaled to the full grid; (d) the oracle's history commit
    arithmetic on the same sample, scaled, and its GND update (the regularised Nye tensor
    of the plastic distortion, a 9-component FFT round trip, and the density) on the full
    grid.  The oracle time of one increment is projected with the operator-application,
    constitutive-call and alternating-pass counts of the GPU FP64 increments (same
    tolerances; the timed increments solve no phase field, so no phase-field Krylov
    iteration enters), and the rate is voxels x operator applications / projected time.
    """
    from oracle import (OracleRVE, momentum_operator, to_mandel2, from_mandel2, return_map,
                        we_plus, nye_tensor, gnd_density)
    from oracle.spectral import WORKERS
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    M = o.grid.M
    gK = (1.0 + w.k_res) * o.tab.C[o.gid]
    matvec, prec, _ = momentum_operator(o.grid, gK)
    x = np.random.default_rng(0).standard_normal(3 * M) * 1e-9
    t0 = time.perf_counter()
    for _ in range(n_apply):
        x = prec(matvec(x))
    t_apply = (time.perf_counter() - t0) / n_apply
    sub = np.arange(0, M, stride)
    eps = np.zeros((len(sub), 3, 3))
    eps[:, 1, 1] = np.sum(inp["deps"][:first + 1])
    t = o.tab
    gid = o.gid[sub]
    t0 = time.perf_counter()
    sig, dgam, _, _ = return_map(to_mandel2(eps), np.zeros((len(sub), 6)), o.g[sub], inp["dt"][0],
                                 t.C[gid], t.S[gid], t.P[gid], law=o.law)
    t_const = (time.perf_counter() - t0) * M / len(sub)
    # phase-field source on the sample (as the oracle's alternating pass computes it)
    t0 = time.perf_counter()
    epsp_tr = from_mandel2(np.einsum("ma,mai->mi", dgam, t.P[gid]))
    tau = np.einsum("mai,mi->ma", t.P[gid], sig)
    wp_tr = (tau * dgam).sum(1)
    we = we_plus(eps - epsp_tr, t.C4[gid])
    Sd = np.where(we + wp_tr > 0.0, w.ell / w.gc_value() * np.maximum(0.0, we + wp_tr), 0.0)
    t_source = (time.perf_counter() - t0) * M / len(sub)
    # history commit on the sample, GND update on the full grid
    t0 = time.perf_counter()
    dbeta = np.einsum("ma,maij->mij", dgam, t.SN[gid])
    rho = o.rho_ssd[sub] + w.lambda_ssd * np.sqrt(2.0 / 3.0 * np.einsum("mij,mij->m", dbeta, dbeta))
    gs = w.xi_store * wp_tr / np.sqrt(rho + o.rho_gnd[sub])
    _ = np.maximum(o.H[sub], we), (gs >= w.G_crit) & (Sd >= 0.0)
    t_commit = (time.perf_counter() - t0) * M / len(sub)
    t0 = time.perf_counter()
    lam = nye_tensor(o.grid, o.beta + 1e-6, w.ell_fp)
    gnd_density(lam, t.R[o.gid], w.burgers)
    t_gnd = time.perf_counter() - t0
    n_mv = np.mean([s["krylov_iters"] for s in gpu_stats])
    n_cs = np.mean([s["newton_iters"] + s["ls_cuts"] + s["stag_iters"] for s in gpu_stats])
    n_st = np.mean([s["stag_iters"] for s in gpu_stats])
    t_inc = n_mv * t_apply + n_cs * t_const + n_st * t_source + t_commit + t_gnd
    return {"value": round(M * n_mv / t_inc, 1), "unit": "voxel-iters/s",
            "cores": int(WORKERS), "cpu_model": _cpu_model(), "kind": "oracle",
            "sample": (f"{n_apply} oracle operator+preconditioner applications on the full "
                       f"{w.name} grid ({t_apply:.2f} s each); the oracle return map "
                       f"({t_const:.1f} s per full-grid call), phase-field source "
                       f"({t_source:.1f} s) and commit arithmetic ({t_commit:.2f} s) on 1/"
                       f"{stride} of its voxels, scaled; its GND update on the full grid "
                       f"({t_gnd:.1f} s); one increment projected with the GPU run's counts "
                       f"({n_mv:.0f} operator applications, {n_cs:.0f} constitutive calls, "
                       f"{n_st:.0f} alternating passes) = {t_inc:.0f} s; scipy.fft with "
                       f"{WORKERS} workers")}


def damage_leg(RVE, precision, torch, w, inp, warmup, steps, gcrit_pow, gc, max_krylov=4000,
               reps=20):
    """The headline increments with the stored-energy threshold G_crit lowered from 4 J/m^2
    by 2^gcrit_pow, so that the threshold is reached in the first increments and the timed
    ones solve the phase field (eqs. phase, precph) with a non-zero driving state, and the
    toughness G_c raised to gc so that the damage grows stably instead of localising into
    a through crack within one increment; the Krylov cap is raised for the stiffness
    contrast of the damaged voxels.  Also times one
    phase-field CG iteration in isolation (HIP events on the library's stream): its
    algorithmic bytes (FP64 vectors, the one-component FFT round trip) over its duration."""
    from paper_2304_01125_amd.rve import PASSES
    wd = dataclasses.replace(w, G_crit=4.0 / 2 ** gcrit_pow, Gc=gc, max_krylov=max_krylov)
    r, dt, kry, stats, _ = run_leg(RVE, precision, wd.desc(), inp, warmup, steps, torch)
    s = r.stream
    r.launch_pass(PASSES["pf_iter"], 2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    nbytes = r.launch_pass(PASSES["pf_iter"], reps)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    r.close()
    pf = int(sum(x["pf_iters"] for x in stats))
    return {"G_crit": wd.G_crit, "Gc": wd.Gc, "value": round(wd.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "krylov_iters": kry, "pf_iters": pf,
            "stag_iters": int(sum(x["stag_iters"] for x in stats)),
            "newton_iters": int(sum(x["newton_iters"] for x in stats)),
            "ms_phase_field": round(sum(x["ms_phase_field"] for x in stats), 2),
            "max_phi": float(max(x["max_phi"] for x in stats)),
            "n_triggered": float(stats[-1]["n_triggered"]),
            "pf_iteration": {"ms": round(ms, 5), "bytes": nbytes,
                             "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                             "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def material_leg(RVE, precision, torch, name="cmsx4-laguerre-128-g512", warmup=2, steps=2):
    """The same increment with the thermally activated flow rule and Taylor hardening
    (Table 1 constants): the first increments stay elastic and serve as warm-up, the
    timed ones yield.  Also times the constitutive kernel at the yielded state."""
    from synth import workload, make_inputs
    from paper_2304_01125_amd.rve import PASSES
    w = workload(name)
    inp = make_inputs(w)
    r, dt, kry, stats, _ = run_leg(RVE, precision, w.desc(), inp, warmup, steps, torch)
    s = r.stream
    r.launch_pass(PASSES["constitutive"], 1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    r.launch_pass(PASSES["constitutive"], 5)
    e1.record(s)
    e1.synchronize()
    r.close()
    return {"workload": name, "flow": "thermally activated (eq. flowrule), Taylor hardening",
            "value": round(w.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "increments": f"{warmup}..{warmup + steps - 1}",
            "krylov_iters": kry, "newton_iters": int(sum(x["newton_iters"] for x in stats)),
            "constitutive_ms": round(e0.elapsed_time(e1) / 5, 4)}


def stress_control_leg(RVE, precision, w, inp, warmup, steps, torch):
    """The headline increments under uniaxial stress: the macro yy strain follows the
    load, every other macro stress component is held at zero (mixed control)."""
    r, dt, kry, stats, macro = run_leg(RVE, precision, w.desc(), inp, warmup, steps, torch,
                                       stress_mask=0b111101)
    r.close()
    lat = np.abs(macro[:, [0, 2, 3, 4, 5]]).max() / np.abs(macro[:, 1]).max()
    return {"control": "uniaxial stress along y (mixed: yy strain, other macro stresses 0)",
            "value": round(w.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "krylov_iters": kry,
            "newton_iters": int(sum(x["newton_iters"] for x in stats)),
            "max_lateral_macro_stress_rel": float(lat)}


def gmres_leg(RVE, precision, w, inp, warmup, steps, torch, m=10):
    """The headline increments with the paper's restarted GMRES(m) instead of CG."""
    desc = dict(w.desc(), krylov=1, gmres_restart=m)
    r, dt, kry, stats, macro = run_leg(RVE, precision, desc, inp, warmup, steps, torch)
    r.close()
    return {"krylov": f"GMRES({m}), left preconditioned", "value": round(w.nvox * kry / dt, 1),
            "unit": "voxel-iters/s", "ms_per_step": round(1e3 * dt / steps, 2),
            "krylov_iters": kry, "newton_iters": int(sum(x["newton_iters"] for x in stats))}


def rotated_leg(RVE, precision, w, inp, warmup, steps, torch):
    """The headline increments with the rotated-scheme discrete derivative."""
    desc = dict(w.desc(), scheme=1)
    r, dt, kry, stats, macro = run_leg(RVE, precision, desc, inp, warmup, steps, torch)
    r.close()
    return {"derivative": "rotated finite differences (gradient, divergence, acoustic tensor)",
            "value": round(w.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "krylov_iters": kry,
            "newton_iters": int(sum(x["newton_iters"] for x in stats))}


def _timed(step, warmup, steps, torch):
    """Warm-up increments, then `steps` timed ones; returns (seconds, Krylov iterations,
    per-increment stats)."""
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step(k) for k in range(warmup, warmup + steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, int(sum(x["krylov_iters"] for x in stats)), stats


def finite_leg(RVE, precision, w, inp, warmup, steps, torch, m=30):
    """The headline grid and load with finite-strain kinematics (F = Fe Fp, first
    Piola-Kirchhoff stress, the 9-component momentum operator; GMRES(m), the solver these
    kinematics run with); the macro deformation gradient's yy entry follows the load."""
    r = RVE(dict(w.desc(), kinematics=1, krylov=1, gmres_restart=m), precision)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])

    def step(k):
        dF = np.zeros(9)
        dF[4] = inp["deps"][k]
        return r.step_finite(dF, inp["dt"][k])
    dt, kry, stats = _timed(step, warmup, steps, torch)
    r.close()
    return {"kinematics": f"finite strain, GMRES({m})", "value": round(w.nvox * kry / dt, 1),
            "unit": "voxel-iters/s (9-component operator)",
            "ms_per_step": round(1e3 * dt / steps, 2), "krylov_iters": kry,
            "newton_iters": int(sum(x["newton_iters"] for x in stats))}


def gnd_leg(RVE, precision, torch, name="cmsx4-laguerre-128-g512", warmup=2, steps=1):
    """The Table 1 material's yielding increments with the Taylor strength coupled to the
    GND density inside the increment (Nye tensor of the trial plastic distortion, resolved
    by the alternating minimisation)."""
    from synth import workload, make_inputs
    w = workload(name)
    inp = make_inputs(w)
    r = RVE(dict(w.desc(), gnd_coupling=1), precision)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    dt, kry, stats = _timed(lambda k: r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k]),
                            warmup, steps, torch)
    r.close()
    return {"workload": name, "hardening": "Taylor, GND-coupled within the increment",
            "value": round(w.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "increments": f"{warmup}..{warmup + steps - 1}",
            "krylov_iters": kry, "newton_iters": int(sum(x["newton_iters"] for x in stats)),
            "stag_iters": int(sum(x["stag_iters"] for x in stats))}


def plate_leg(RVE, precision, torch, warmup=1, steps=4):
    """A plate of 256 x 256 x 1 voxels (the paper's plate grids) with 64 Voronoi grains in
    pointwise plane stress under uniaxial load: yy strain controlled, the in-plane xx and
    xy macro stresses held at zero."""
    from synth import workload, make_inputs
    w = workload("plate-256-g64")
    inp = make_inputs(w)
    r = RVE(dict(w.desc(), plane_stress=1), precision)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    dt, kry, stats = _timed(lambda k: r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k],
                                             dsig6=np.zeros(6), stress_mask=0b100001),
                            warmup, steps, torch)
    r.close()
    return {"workload": w.name, "grid": list(w.n), "grains": w.n_grains,
            "control": "plane stress, uniaxial (yy strain; xx, xy macro stress 0)",
            "value": round(w.nvox * kry / dt, 1), "unit": "voxel-iters/s",
            "ms_per_step": round(1e3 * dt / steps, 2), "krylov_iters": kry,
            "newton_iters": int(sum(x["newton_iters"] for x in stats))}


def _guarded(fn, *args, **kw):
    """A widened leg's failure is reported in its own entry; it does not end the run."""
    try:
        return fn(*args, **kw)
    except Exception as e:           # noqa: BLE001 - recorded, not raised
        return {"error": f"{type(e).__name__}: {e}"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    serve_items = None
    if a.serve_requests > 0:     # the serving requests' inputs, before any GPU work
        from paper_2304_01125_amd.serve import prepare
        from synth import serving_requests
        serve_items = prepare(serving_requests(a.serve_requests, 4)[2],
                              min(16, os.cpu_count() or 1))
    import torch
    from paper_2304_01125_amd import RVE, RVE_FP64, RVE_MIXED
    from synth import workload, make_inputs

    w = workload(a.workload)
    inp = make_inputs(w)
    desc = dict(w.desc(), scheme=1 if a.deriv == "rotated" else 0)
    r64, dt64, kry64, st64, macro64 = run_leg(RVE, RVE_FP64, desc, inp, a.warmup, a.steps, torch,
                                              live=True)
    value = w.nvox * kry64 / dt64
    passes = time_passes(r64, torch, a.pass_reps)
    # dominant kernel of the operator as the solver runs it: largest share of one matvec
    if "zgrad" in passes:
        per_mv = {"zgrad": 1, "fft_y": 2, "x_tangent": 1, "zdiv": 1}
    else:
        per_mv = {"fft_z": 2, "fft_y": 2, "x_tangent": 1, "grad": 1, "div": 1}
    dom = max(per_mv, key=lambda k: per_mv[k] * passes[k]["ms"])
    d = passes[dom]
    # the dominant kernel (the row tangent pass) timed live inside the timed increments:
    # HIP events on the library's stream around its launch in every LIVE_EVERY-th CG
    # iteration (the same kernel on the same data each time)
    n_live, ms_live = r64.live
    avg = ms_live / n_live if (dom == "x_tangent" and n_live) else d["ms"]
    gbs = d["bytes"] / (avg * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, w.n[0]),
            "avg_launch_ms": round(avg, 5), "bytes_per_launch": d["bytes"],
            "timed_launches": n_live if dom == "x_tangent" else 0}
    r64.close()
    out = {"metric": METRIC, "value": round(value, 1), "unit": "voxel-iters/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * dt64 / a.steps, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w.name, "grid": list(w.n), "grains": w.n_grains,
                      "derivative": a.deriv,
                      "load": f"R={w.ratio}, +-{w.amplitude * 100:.1f}%, increments "
                              f"{a.warmup}..{a.warmup + a.steps - 1}",
                      "tolerances": {"lin": w.tol_lin, "newton": w.tol_newton,
                                     "stag": w.tol_stag}},
           "krylov_iters": kry64,
           "passes": {k: {"ms": round(v["ms"], 5), "GB/s": round(v["gbs"], 1)}
                      for k, v in passes.items()},
           "roofline": roof}
    if not a.no_mixed:
        r32, dt32, kry32, st32, macro32 = run_leg(RVE, RVE_MIXED, desc, inp, a.warmup, a.steps,
                                                  torch)
        p32 = time_passes(r32, torch, a.pass_reps)
        r32.close()
        err = np.abs(macro32 - macro64).max(axis=1) / np.abs(macro64).max(axis=1)
        out["mixed"] = {"value": round(w.nvox * kry32 / dt32, 1), "unit": "voxel-iters/s",
                        "ms_per_step": round(1e3 * dt32 / a.steps, 2), "dtype": "f32+f64",
                        "krylov_iters": kry32,
                        "macro_stress_rel_err_vs_fp64": float(err.max()),
                        "passes": {k: {"ms": round(v["ms"], 5), "GB/s": round(v["gbs"], 1)}
                                   for k, v in p32.items()}}
    if not a.no_gmres:
        out["gmres"] = gmres_leg(RVE, RVE_FP64, w, inp, a.warmup, a.steps, torch,
                                 a.gmres_restart)
    if not a.no_rotated and a.deriv == "spectral":
        out["rotated"] = rotated_leg(RVE, RVE_FP64, w, inp, a.warmup, a.steps, torch)
    if not a.no_stress_control:
        out["stress_control"] = stress_control_leg(RVE, RVE_FP64, w, inp, a.warmup, a.steps, torch)
    if not a.no_damage:
        out["damage"] = damage_leg(RVE, RVE_FP64, torch, w, inp, a.warmup, a.steps,
                                   a.damage_gcrit_pow, a.damage_gc)
    if not a.no_material:
        out["material"] = material_leg(RVE, RVE_FP64, torch)
    if not a.no_finite:
        out["finite_strain"] = _guarded(finite_leg, RVE, RVE_FP64, w, inp, a.warmup, a.steps,
                                        torch)
    if not a.no_gnd:
        out["gnd_coupled"] = _guarded(gnd_leg, RVE, RVE_FP64, torch)
    if not a.no_plate:
        out["plane_stress"] = _guarded(plate_leg, RVE, RVE_FP64, torch)
    if a.serve_requests > 0:
        from paper_2304_01125_amd.serve import serve_benchmark
        out["serving"] = serve_benchmark(a.serve_requests, a.serve_slots, 4, log=lambda m: print(
            "# " + m, file=sys.stderr, flush=True), items=serve_items)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, inp, st64, a.warmup)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
