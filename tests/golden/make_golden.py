"""Writes the stored expected values of the GPU parity tests by running the CPU oracle.

Only ``oracle`` (and the seeded input generators in ``synth``) are called.  Outputs:

* notched16.npz -- the notched single crystal on 16^3 (the plain-method FP64 workload),
  tight (parity) tolerances, fields after selected increments and the macro stress of
  every increment, up to the first increment where the damage jumps by more than 0.5
  in one increment or the alternating-minimisation count exceeds three times its
  median (beyond that the crack path may bifurcate and several answers are correct).
* voronoi64.npz -- the 64^3 Voronoi polycrystal (64 grains), tight tolerances, every
  increment up to two increments past damage initiation (G_crit lowered by a power of 2
  so that it initiates early, as the workload records), fields at 4096 seeded sample voxels
  after increment 1 and the last two, the macro stress, maximum damage and number of
  triggered voxels of each.
* cmsx4_16.npz -- the 16^3 four-grain polycrystal with the thermally activated flow
  rule and Taylor hardening (Table 1 constants), tight tolerances, the first six
  increments (elastic, then yielding): every field after increments 3 and 5, macro stress
  and iteration counts of each.
* finite16.npz -- the 16^3 eight-grain polycrystal in finite strain (F = Fe Fp, first
  Piola-Kirchhoff stress), tight tolerances, uniaxial strain along y, four yielding
  increments: every field after increments 1 and 3, the macro first Piola-Kirchhoff stress
  of each.

Usage: python tests/golden/make_golden.py [notched16|voronoi64|cmsx4_16|finite16] ...
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import OracleRVE          # noqa: E402
from oracle.finite import OracleFiniteRVE   # noqa: E402
from synth import workload, make_inputs, small_polycrystal   # noqa: E402

FIELDS = ("strain", "stress", "damage", "gs", "wp", "rho_gnd")
FIELDS_CMSX4 = FIELDS + ("rho_ssd", "g", "eps_p")
FIELDS64 = FIELDS + ("h", "wcrit", "trig")


def notched16(max_inc=40, snaps=(5, 11, 13, 15, 19, 25, 31, 39)):
    w = workload("notched-crystal-16").parity()
    inp = make_inputs(w)
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    out = {"macro_stress": [], "stag": [], "max_phi_slip": []}
    stags = []
    prev_phi = o.phi.copy()
    notch = inp["phi0"] >= 1.0
    t0 = time.time()
    last = -1
    for k in range(max_inc):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        jump = np.abs(o.phi - prev_phi)[~notch].max()
        prev_phi = o.phi.copy()
        stags.append(st["stag"])
        print(f"inc {k}: {time.time() - t0:.0f}s stag {st['stag']} newton {st['newton']} "
              f"jump {jump:.3f} maxphi {o.phi[~notch].max():.4f}", flush=True)
        if jump > 0.5 or (k > 4 and st["stag"] > 3 * max(2, np.median(stags))):
            # keep the increment of the jump itself as a separate record, then stop
            print("stopping: damage instability", flush=True)
            f = o.fields()
            for name in FIELDS:
                out[f"jump_{name}"] = f[name]
            out["jump_inc"] = k
            out["jump_macro_stress"] = st["macro_stress"]
            np.savez_compressed(os.path.join(HERE, "notched16.npz"), last=last,
                                **{k2: np.asarray(v) for k2, v in out.items()})
            break
        last = k
        out["macro_stress"].append(st["macro_stress"])
        out["stag"].append(st["stag"])
        out["max_phi_slip"].append(float(o.phi[~notch].max()))
        if k in snaps:
            f = o.fields()
            for name in FIELDS:
                out[f"inc{k}_{name}"] = f[name]
        np.savez_compressed(os.path.join(HERE, "notched16.npz"), last=last,
                            **{k2: np.asarray(v) for k2, v in out.items()})


def voronoi64(max_inc=16, n_sample=4096, keep=2, stop_after=1):
    """Config 1 up to damage initiation: increments until the damage has been non-zero for
    `stop_after` increments (at most max_inc), the macro stress, the maximum damage and the
    number of triggered voxels of each, and sampled fields after increment 1 and the last
    `keep` increments.  (The first damaging increment needs about 50 alternating passes at
    the parity tolerances, about two hours of this oracle on 8 cores; the next one, where
    the damage runs to 1, about 100.)"""
    w = workload("voronoi-64-g64").parity()
    inp = make_inputs(w)
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    idx = np.sort(np.random.default_rng(64).choice(w.nvox, n_sample, replace=False))
    out = {"sample": idx, "macro_stress": [], "max_phi": [], "n_trig": [], "stag": []}
    t0 = time.time()
    damaged = 0
    for k in range(max_inc):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        print(f"inc {k}: {time.time() - t0:.0f}s newton {st['newton']} matvecs {st['matvecs']} "
              f"stag {st['stag']} n_trig {st['n_trig']} max phi {st['max_phi']:.3e}", flush=True)
        out["macro_stress"].append(st["macro_stress"])
        out["max_phi"].append(st["max_phi"])
        out["n_trig"].append(st["n_trig"])
        out["stag"].append(st["stag"])
        damaged += st["max_phi"] > 0.0
        f = o.fields()
        for name in FIELDS64:
            out[f"inc{k}_{name}"] = f[name][idx]
        drop = k - keep                  # keep increment 1 and the latest `keep` increments
        if drop >= 0 and drop != 1:
            for name in FIELDS64:
                out.pop(f"inc{drop}_{name}", None)
        np.savez_compressed(os.path.join(HERE, "voronoi64.npz"), last=k, G_crit=w.G_crit,
                            **{k2: np.asarray(v) for k2, v in out.items()})
        if damaged >= stop_after:
            break


def cmsx4_16(n_inc=6, snaps=(3, 5)):
    w = workload("cmsx4-voronoi-16-g4").parity()
    inp = make_inputs(w)
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    out = {"macro_stress": [], "newton": [], "stag": []}
    t0 = time.time()
    for k in range(n_inc):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        print(f"inc {k}: {time.time() - t0:.0f}s stag {st['stag']} newton {st['newton']}",
              flush=True)
        out["macro_stress"].append(st["macro_stress"])
        out["newton"].append(st["newton"])
        out["stag"].append(st["stag"])
        if k in snaps:
            f = o.fields()
            for name in FIELDS_CMSX4:
                out[f"inc{k}_{name}"] = f[name]
    np.savez_compressed(os.path.join(HERE, "cmsx4_16.npz"), last=n_inc - 1,
                        **{k2: np.asarray(v) for k2, v in out.items()})


FIELDS_FINITE = ("defgrad", "pk1", "fp", "damage", "gs", "wp", "rho_ssd", "rho_gnd", "g", "h")


def finite_workload():
    """The finite-strain parity workload (also built by the GPU test)."""
    return small_polycrystal(n=16, n_grains=8, seed=7).parity()


def finite16(n_inc=4, snaps=(1, 3)):
    w = finite_workload()
    inp = make_inputs(w)
    o = OracleFiniteRVE(dict(w.desc(), kinematics=1), inp["grain"], inp["quat"], inp["tau_c0"],
                        inp["phi0"])
    out = {"macro_pk1": [], "newton": []}
    t0 = time.time()
    for k in range(n_inc):
        dF = np.zeros(9)
        dF[4] = inp["deps"][k]
        st = o.step(dF, inp["dt"][k])
        print(f"inc {k}: {time.time() - t0:.0f}s newton {st['newton']}", flush=True)
        out["macro_pk1"].append(st["macro_stress"])
        out["newton"].append(st["newton"])
        if k in snaps:
            f = o.fields()
            for name in FIELDS_FINITE:
                out[f"inc{k}_{name}"] = f[name]
    np.savez_compressed(os.path.join(HERE, "finite16.npz"), last=n_inc - 1,
                        **{k2: np.asarray(v) for k2, v in out.items()})


def laguerre128(n_inc=5, n_sample=4096):
    """The benchmark workload (128^3, 512 Laguerre grains) at the paper's production
    tolerances: macro stress, Newton and alternating counts of its first n_inc increments and
    sampled strain and stress after the first, the reference the GPU's FP64 and mixed
    precision increments are compared with at full size (about 20 minutes per increment of
    this oracle on 8 cores)."""
    w = workload("laguerre-128-g512")
    inp = make_inputs(w)
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    idx = np.sort(np.random.default_rng(128).choice(w.nvox, n_sample, replace=False))
    out = {"sample": idx, "macro_stress": [], "newton": [], "stag": []}
    t0 = time.time()
    for k in range(n_inc):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
        print(f"inc {k}: {time.time() - t0:.0f}s newton {st['newton']} matvecs {st['matvecs']} "
              f"stag {st['stag']}", flush=True)
        out["macro_stress"].append(st["macro_stress"])
        out["newton"].append(st["newton"])
        out["stag"].append(st["stag"])
        if k == 0:
            f = o.fields()
            for name in ("strain", "stress"):
                out[f"inc0_{name}"] = f[name][idx]
        np.savez_compressed(os.path.join(HERE, "laguerre128.npz"), last=k,
                            **{k2: np.asarray(v) for k2, v in out.items()})


def plate256(n_inc=6, n_sample=4096):
    """The paper's plate grid (256 x 256 x 1, 64 grains) in pointwise plane stress under
    uniaxial load (yy strain controlled, xx and xy macro stress zero) at the production
    tolerances: macro stress, Newton and alternating counts of its first n_inc increments,
    and sampled strain and stress after the first and the last."""
    w = workload("plate-256-g64")
    inp = make_inputs(w)
    d = dict(w.desc(), plane_stress=1)
    o = OracleRVE(d, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    idx = np.sort(np.random.default_rng(256).choice(w.nvox, n_sample, replace=False))
    out = {"sample": idx, "macro_stress": [], "macro_strain": [], "newton": [], "stag": []}
    t0 = time.time()
    for k in range(n_inc):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), 0b100001)
        print(f"inc {k}: {time.time() - t0:.0f}s newton {st['newton']} stag {st['stag']}",
              flush=True)
        out["macro_stress"].append(st["macro_stress"])
        out["macro_strain"].append(st["macro_strain"])
        out["newton"].append(st["newton"])
        out["stag"].append(st["stag"])
        if k in (0, n_inc - 1):
            f = o.fields()
            for name in ("strain", "stress"):
                out[f"inc{k}_{name}"] = f[name][idx]
    np.savez_compressed(os.path.join(HERE, "plate256.npz"), last=n_inc - 1,
                        **{k2: np.asarray(v) for k2, v in out.items()})


if __name__ == "__main__":
    for name in sys.argv[1:] or ["notched16", "voronoi64", "cmsx4_16", "finite16"]:
        globals()[name]()
