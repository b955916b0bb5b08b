"""Parity at the full sizes of the benchmark workloads: the 128^3 polycrystal with 512
log-normal Laguerre grains (the benchmark's), the 256^3 Voronoi polycrystal with 4096 grains
and 5 % hard grains, and a 512 x 512 x 16 plate-like polycrystal whose fused divergence pass
writes more block partials (49152) than any other grid, on the kernels the benchmark times
(fused z passes, register FFTs, row tangent passes of 128, 256 and 512 points).  A whole
oracle solve at these sizes is too slow for a test, so the first increment is checked on
what the oracle can compute voxel by voxel and on properties that hold at any size:

* the imposed macroscopic strain is the mean strain;
* at 4096 sampled voxels, the GPU stress, slip increments (through eps_p) and slip
  resistance equal the oracle's return map at the GPU strain (state at t = 0 is known);
* the degraded stress is equilibrated: its Fourier divergence i xi~ . sigma^ vanishes;
* the strain is compatible: the oracle's Green projection onto symmetric gradients of
  periodic displacements, sym(i xi~ (x) u^) with u^ = -[xi~.K0.xi~]^-1 i xi~.(K0 : e^) for
  an isotropic reference K0, reproduces the fluctuation e = eps - eps_bar;
* the mixed-precision increment reproduces the FP64 macroscopic stress within 1e-4.
"""
import dataclasses

import numpy as np
import pytest

from synth import workload, make_inputs, small_polycrystal

pytestmark = pytest.mark.gpu
NAME = "laguerre-128-g512"


def _first_increment(precision, parity=True, w=None):
    from paper_2304_01125_amd import RVE
    w = workload(NAME) if w is None else w
    if parity:
        w = w.parity()
    inp = make_inputs(w)
    r = RVE(w.desc(), precision)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    st = r.step([0, inp["deps"][0], 0, 0, 0, 0], inp["dt"][0])
    print(f"  {w.name} precision {precision}: newton {st['newton_iters']} krylov "
          f"{st['krylov_iters']} stag {st['stag_iters']}", flush=True)
    return w, inp, r, st


def _compatibility_error(grid, strain, ebar):
    """max |P(e^) - e^| / max |e^| over the spectrum of e = eps - eps_bar, with P the
    oracle's projection onto compatible strains (isotropic reference medium)."""
    from oracle.increment import from_tensor6
    from oracle.crystal import cubic_stiffness
    eh = grid.fft(grid.to_grid(from_tensor6(strain - ebar[None])))
    K0 = cubic_stiffness(3.0, 1.0, 1.0)               # isotropic: C44 = (C11 - C12) / 2
    uh = -np.einsum("...ik,...k->...i", grid.acoustic_inverse(K0),
                    grid.div_hat(np.einsum("ijkl,...kl->...ij", K0, eh)))
    del eh
    ph = grid.sym_grad_hat(uh)
    eh = grid.fft(grid.to_grid(from_tensor6(strain - ebar[None])))
    return np.abs(ph - eh).max() / np.abs(eh).max()


def _check_first_increment(w, inp, r, n_sample=4096, seed=11):
    from oracle import GrainTables, return_map, to_mandel2, Grid
    from oracle.increment import from_tensor6
    f = r.fields(("strain", "stress", "stress_eff", "eps_p", "g", "damage"))
    N = w.nvox
    # imposed macro strain
    ebar = np.array([0.0, inp["deps"][0], 0.0, 0.0, 0.0, 0.0])
    assert np.abs(f["strain"].mean(0) - ebar).max() <= 1e-15
    assert np.abs(f["damage"]).max() == 0.0
    # sampled voxels against the oracle's return map at the GPU strain
    idx = np.random.default_rng(seed).choice(N, n_sample, replace=False)
    tab = GrainTables(inp["quat"], w.C11, w.C12, w.C44)
    gid = inp["grain"][idx]
    g0 = np.asarray(inp["tau_c0"])[gid]
    epsM = to_mandel2(from_tensor6(f["strain"][idx]))
    sig, dgam, K, _ = return_map(epsM, np.zeros_like(epsM), g0, inp["dt"][0], tab.C[gid],
                                 tab.S[gid], tab.P[gid], w.gdot0, w.n_exp)
    sig_gpu = to_mandel2(from_tensor6(f["stress_eff"][idx]))
    e_sig = np.linalg.norm(sig_gpu - sig) / np.linalg.norm(sig)
    epsp_o = np.einsum("ma,mai->mi", dgam, tab.P[gid])
    epsp_g = to_mandel2(from_tensor6(f["eps_p"][idx]))
    e_ep = np.linalg.norm(epsp_g - epsp_o) / np.linalg.norm(epsp_o)
    g1 = g0 + w.h_lin * np.abs(dgam).sum(1)
    e_g = np.abs(f["g"][idx] - g1).max() / g1.max()
    print(f"  sampled voxels: stress {e_sig:.2e}, eps_p {e_ep:.2e}, g {e_g:.2e}", flush=True)
    assert np.abs(dgam).max() > 1e-5           # yielding voxels among the samples
    assert e_sig <= 1e-10 and e_ep <= 1e-8 and e_g <= 1e-12
    # equilibrium of the degraded stress
    grid = Grid(w.n, w.h)
    stress = f.pop("stress")
    sh = grid.fft(grid.to_grid(from_tensor6(stress)))
    del stress
    div = np.abs(grid.div_hat(sh)).max() / (np.abs(sh).max() * np.abs(grid.xit).max())
    del sh
    print(f"  equilibrium: max |i xi~ . sigma^| / (max |sigma^| max |xi~|) = {div:.2e}", flush=True)
    assert div <= 1e-9
    # compatibility of the strain
    comp = _compatibility_error(grid, f["strain"], ebar)
    print(f"  compatibility: max |P e^ - e^| / max |e^| = {comp:.2e}", flush=True)
    assert comp <= 1e-12


def test_first_increment_at_full_size_matches_oracle_on_sampled_voxels():
    from paper_2304_01125_amd import RVE_FP64
    w, inp, r, st = _first_increment(RVE_FP64)
    _check_first_increment(w, inp, r)
    r.close()


def test_first_increment_at_256_matches_oracle_on_sampled_voxels():
    """The 256^3 workload (4096 Voronoi grains, 5 % hard grains) in FP64 at parity
    tolerances: the 256-point fused z passes and row tangent pass."""
    from paper_2304_01125_amd import RVE_FP64
    w, inp, r, st = _first_increment(RVE_FP64, w=workload("voronoi-256-g4096-hard"))
    _check_first_increment(w, inp, r, seed=12)
    r.close()


def test_widest_divergence_partials_grid():
    """512 x 512 x 16 (49152 divergence-pass partials, past the CG step's partials before
    their offset was sized from the grid): a full CG solve at parity tolerances."""
    from paper_2304_01125_amd import RVE_FP64
    w = dataclasses.replace(small_polycrystal(n=(512, 512, 16), n_grains=64, seed=13),
                            amplitude=0.005, ratio=-1, cycles=2, incs_per_cycle=20)
    w, inp, r, st = _first_increment(RVE_FP64, w=w)
    _check_first_increment(w, inp, r, seed=13)
    r.close()


def test_mixed_precision_at_full_size_reproduces_fp64_macro_stress():
    from paper_2304_01125_amd import RVE_FP64, RVE_MIXED
    ms = {}
    fields = {}
    for prec in (RVE_FP64, RVE_MIXED):
        w, inp, r, st = _first_increment(prec, parity=False)
        ms[prec] = np.array(st["macro_stress"])
        fields[prec] = r.fields(("stress",))["stress"]
        r.close()
    err = np.abs(ms[RVE_MIXED] - ms[RVE_FP64]).max() / np.abs(ms[RVE_FP64]).max()
    e_field = np.linalg.norm(fields[RVE_MIXED] - fields[RVE_FP64]) / np.linalg.norm(fields[RVE_FP64])
    print(f"  mixed vs FP64: macro stress {err:.2e}, stress field rel. L2 {e_field:.2e}", flush=True)
    assert err <= 1e-4


def test_uniaxial_stress_at_full_size():
    """Mixed control at the benchmark size: the first increment under uniaxial stress at
    parity tolerances; the lateral macro stresses vanish, the yy macro strain is the
    imposed one, the degraded stress is equilibrated, and at 4096 sampled voxels the GPU
    stress equals the oracle's return map at the GPU strain."""
    from oracle import GrainTables, return_map, to_mandel2, Grid
    from oracle.increment import from_tensor6
    from paper_2304_01125_amd import RVE, RVE_FP64
    w = workload(NAME).parity()
    inp = make_inputs(w)
    r = RVE(w.desc(), RVE_FP64)
    r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    st = r.step([0, inp["deps"][0], 0, 0, 0, 0], inp["dt"][0], dsig6=np.zeros(6),
                stress_mask=0b111101)
    ms, me = np.array(st["macro_stress"]), np.array(st["macro_strain"])
    print(f"  uniaxial stress: newton {st['newton_iters']} krylov {st['krylov_iters']}, "
          f"macro stress {ms.tolist()}, macro strain {me.tolist()}", flush=True)
    assert np.abs(ms[[0, 2, 3, 4, 5]]).max() <= 1e-9 * abs(ms[1])
    assert abs(me[1] - inp["deps"][0]) <= 1e-15
    f = r.fields(("strain", "stress", "stress_eff"))
    r.close()
    assert np.abs(f["strain"].mean(0) - me).max() <= 1e-15
    idx = np.random.default_rng(12).choice(w.nvox, 4096, replace=False)
    tab = GrainTables(inp["quat"], w.C11, w.C12, w.C44)
    gid = inp["grain"][idx]
    g0 = np.asarray(inp["tau_c0"])[gid]
    epsM = to_mandel2(from_tensor6(f["strain"][idx]))
    sig, _, _, _ = return_map(epsM, np.zeros_like(epsM), g0, inp["dt"][0], tab.C[gid],
                              tab.S[gid], tab.P[gid], w.gdot0, w.n_exp)
    e_sig = np.linalg.norm(to_mandel2(from_tensor6(f["stress_eff"][idx])) - sig) / np.linalg.norm(sig)
    grid = Grid(w.n, w.h)
    sh = grid.fft(grid.to_grid(from_tensor6(f["stress"])))
    div = np.abs(grid.div_hat(sh)).max() / (np.abs(sh).max() * np.abs(grid.xit).max())
    print(f"  sampled voxels: stress {e_sig:.2e}; equilibrium {div:.2e}", flush=True)
    assert e_sig <= 1e-10 and div <= 1e-9



def test_benchmark_increments_match_stored_oracle_at_production_tolerances():
    """The benchmark workload (128^3, 512 Laguerre grains) at the paper's tolerances in FP64
    and in mixed precision against the stored oracle run of the same increments
    (tests/golden/make_golden.py laguerre128): the macro stress of every stored increment
    (mixed: the 1e-4 of the precision target; FP64: 1e-5, the same solver path with the
    same Newton and Krylov counts, so rounding apart, observed 3e-14 on the first
    increment; the bar leaves room for a Krylov solve that stops one iteration apart) and
    the sampled strain and stress after the first."""
    import os
    from paper_2304_01125_amd import RVE, RVE_FP64, RVE_MIXED
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "laguerre128.npz")
    ref = np.load(path)
    last = int(ref["last"])
    w = workload("laguerre-128-g512")
    inp = make_inputs(w)
    idx = ref["sample"]
    worst = {}
    for prec, bar in ((RVE_FP64, 1e-5), (RVE_MIXED, 1e-4)):
        r = RVE(w.desc(), prec)
        r.set_microstructure(inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
        errs = []
        for k in range(last + 1):
            st = r.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
            ms = np.array(st["macro_stress"])
            e = np.abs(ms - ref["macro_stress"][k]).max() / np.abs(ref["macro_stress"][k]).max()
            errs.append(e)
            print(f"  precision {prec} inc {k}: newton {st['newton_iters']} (oracle "
                  f"{int(ref['newton'][k])}) krylov {st['krylov_iters']} macro stress {e:.2e}",
                  flush=True)
            if k == 0:
                f = r.fields(("strain", "stress"))
                for name in ("strain", "stress"):
                    a, b = f[name][idx], ref[f"inc0_{name}"]
                    fe = np.linalg.norm(a - b) / np.linalg.norm(b)
                    print(f"    inc 0 {name} at {len(idx)} sampled voxels: {fe:.2e}", flush=True)
                    assert fe <= bar, (prec, name, fe)
        r.close()
        worst[prec] = max(errs)
        assert worst[prec] <= bar, (prec, worst[prec])
    print("  worst macro stress error:", worst, flush=True)
