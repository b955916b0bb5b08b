"""Pins of the oracle's thermally activated flow rule (eq. flowrule) and Taylor hardening
(Sec. 2.1, Table 1), independent of the oracle's own formulas where the mathematics
allows: the elastic range, sinh at a chosen argument, the rate-independent (Schmid)
limit in closed form, a single active system solved as a scalar equation by bisection,
finite differences of the tangent and energy, symmetry, and a homogeneous crystal whose
increment reduces to one material point."""
import numpy as np
from scipy.optimize import brentq

from oracle import GrainTables, return_map, DunneLaw, OracleRVE, to_mandel2
from synth import shoemake_quaternions, small_polycrystal, cmsx4, make_inputs, Workload

W = Workload(name="pins", n=(8, 8, 8), n_grains=1, seed=0, cycles=1,
             incs_per_cycle=20, **cmsx4())
D = W.desc()


def _law(dV=None):
    return DunneLaw(D["rho_m"], D["burgers"], D["v_D"], D["dF"], D["k_B"], D["T"],
                    D["dV"] if dV is None else dV)


def _tables(seed):
    return GrainTables(shoemake_quaternions(1, np.random.default_rng(seed)), D["C11"], D["C12"],
                       D["C44"])


def test_table1_constants_in_si_units():
    # Table 1 prints b in mm, rho_m and lambda in mm^-2, elastic constants in GPa and the
    # initial CRSS in MPa
    assert np.isclose(D["burgers"], 3.5e-7 * 1e-3)
    assert np.isclose(D["rho_m"], 5.0e6 * 1e6)
    assert np.isclose(D["lambda_ssd"], 150e6 * 1e6)
    assert (D["C11"], D["C12"], D["C44"]) == (250e9, 161e9, 129e9)
    assert D["tau_c0"] == 350e6 and D["v_D"] == 1e11 and D["T"] == 295.0
    assert D["k_B"] == 1.4e-23 and D["dF"] == 4.9e-20
    # A = rho_m b^2 v_D exp(-dF/kT): 5e12 * 1.225e-19 * 1e11 * exp(-11.86440677966...)
    law = _law()
    assert abs(law.A - 0.430982561068905) <= 1e-12
    assert abs(law.beta * 4.13e-21 - 20 * (3.5e-10) ** 3) <= 1e-12 * 20 * (3.5e-10) ** 3


def test_slip_increment_at_chosen_arguments():
    law = _law()
    g = np.array([400e6])
    dt = 2.0
    # beta <|tau| - g> = ln(1 + sqrt 2), where sinh = 1 and cosh = sqrt 2
    o = np.log1p(np.sqrt(2.0)) / law.beta
    tau = np.array([[g[0] + o, -(g[0] + o), 0.5 * g[0], -g[0], g[0] + 1e-30]])
    dg, ddg = law.increments(tau, g, dt)
    assert np.allclose(dg[0, :2], [dt * law.A, -dt * law.A], rtol=1e-14)
    assert np.allclose(ddg[0, :2], dt * law.A * law.beta * np.sqrt(2.0), rtol=1e-14)
    # no slip up to the threshold (the printed sinh would be negative there)
    assert np.all(dg[0, 2:] == 0.0) and np.all(ddg[0, 2:4] == 0.0)
    # the potential is the integral of the slip increment along tau
    taus = np.linspace(g[0], g[0] + 3 * o, 20001)
    F = law.potential(taus[:, None], np.full(len(taus), g[0]), dt)
    dgs = law.increments(taus[:, None], np.full(len(taus), g[0]), dt)[0][:, 0]
    trap = np.concatenate([[0.0], np.cumsum(0.5 * (dgs[1:] + dgs[:-1]) * np.diff(taus))])
    assert np.abs(F - trap).max() <= 1e-7 * F[-1]


def test_elastic_below_the_critical_resolved_shear_stress():
    t = _tables(4)
    eps = to_mandel2(np.array([[[1e-3, 1e-4, 0], [1e-4, -5e-4, 2e-4], [0, 2e-4, 3e-4]]]))
    g = np.array([1e9])
    sig, dg, K, _ = return_map(eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=_law())
    tau = t.P[0] @ sig[0]
    assert np.abs(tau).max() < g[0]
    assert np.all(dg == 0.0)
    assert np.allclose(sig[0], t.C[0] @ eps[0], rtol=1e-14)
    assert np.allclose(K[0], t.C[0], rtol=1e-13)


def _single_system(seed, dV=None):
    t = _tables(seed)
    P1 = t.P[:, :1, :]
    p = P1[0, 0]
    # strain along C^-1 p: the trial stress is a pure resolved shear on the kept system
    eps = (2.5 * D["tau_c0"] / (p @ p)) * (t.S[0] @ p)[None]
    return t, P1, p, eps


def test_single_system_reduces_to_scalar_equation():
    t, P1, p, eps = _single_system(9)
    law = _law()
    g = np.array([D["tau_c0"]])
    dt = 2.0
    sig, dg, K, _ = return_map(eps, np.zeros((1, 6)), g, dt, t.C, t.S, P1, law=law)
    tau_tr = p @ t.C[0] @ eps[0]
    pcp = p @ t.C[0] @ p
    f = lambda tau: tau - tau_tr + pcp * dt * law.A * np.sinh(law.beta * (tau - g[0]))
    tau = brentq(f, g[0], tau_tr, xtol=1e-16 * tau_tr, rtol=1e-15, maxiter=500)
    assert abs(p @ sig[0] - tau) <= 1e-12 * tau
    assert tau_tr > 2 * g[0] and dg[0, 0] > 0


def test_rate_independent_limit_is_schmid_single_slip():
    # a large activation volume makes the overstress vanish: tau -> g and
    # dgamma = (tau_tr - g) / (P : C : P) in closed form
    t, P1, p, eps = _single_system(13)
    g = np.array([D["tau_c0"]])
    law = _law(dV=2e4 * D["burgers"] ** 3)
    sig, dg, _, _ = return_map(eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, P1, law=law)
    tau_tr = p @ t.C[0] @ eps[0]
    pcp = p @ t.C[0] @ p
    dg_exact = (tau_tr - g[0]) / pcp
    over = np.arcsinh(dg_exact / (2.0 * law.A)) / law.beta       # the remaining overstress
    assert abs(p @ sig[0] - g[0]) <= 1.01 * over
    assert over <= 1e-5 * g[0]
    assert abs(dg[0, 0] - dg_exact) <= 1.01 * over / pcp


def _plastic(seed):
    t = _tables(seed)
    eps = to_mandel2(np.array([[[0.0, 0, 0], [0, 1.2e-2, 0], [0, 0, -2e-3]]]))
    return t, np.array([395e6]), eps


def test_tangent_and_energy_against_finite_differences():
    t, g, eps = _plastic(7)
    law = _law()
    sig, dgam, K, w = return_map(eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law)
    assert np.abs(dgam).max() > 1e-4
    h = 1e-10
    Kfd = np.zeros((6, 6))
    gfd = np.zeros(6)
    for b in range(6):
        ep = eps[0].copy(); ep[b] += h
        em = eps[0].copy(); em[b] -= h
        sp, _, _, wp = return_map(ep[None], np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law,
                                  sig0=sig)
        sm, _, _, wm = return_map(em[None], np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law,
                                  sig0=sig)
        Kfd[:, b] = (sp[0] - sm[0]) / (2 * h)
        gfd[b] = (wp[0] - wm[0]) / (2 * h)
    assert np.abs(Kfd - K[0]).max() <= 1e-5 * np.abs(K[0]).max()
    assert np.abs(gfd - sig[0]).max() <= 1e-5 * np.abs(sig[0]).max()
    assert np.all(np.linalg.eigvalsh(K[0]) > 0)


def test_root_is_unique_odd_and_dissipative():
    t, g, eps = _plastic(11)
    law = _law()
    a = return_map(eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law)
    b = return_map(eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law,
                   sig0=3.0 * (t.C[0] @ eps[0])[None])
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * np.abs(a[0]).max()
    c = return_map(-eps, np.zeros((1, 6)), g, 2.0, t.C, t.S, t.P, law=law)
    assert np.abs(a[0] + c[0]).max() <= 1e-13 * np.abs(a[0]).max()
    tau = t.P[0] @ a[0][0]
    assert np.all(tau * a[1][0] >= 0.0) and (tau * a[1][0]).sum() > 0


def test_homogeneous_crystal_is_one_material_point_with_taylor_strength():
    # one grain, no notch: every field is uniform, the curl of the plastic distortion
    # vanishes (rho_GND = 0) and each increment is the material-point update at the
    # macroscopic strain with g = tau_c0 + mu b sqrt(rho_SSD)
    w = small_polycrystal(n=8, n_grains=1, seed=21, cycles=1, incs_per_cycle=20,
                          **cmsx4()).parity()
    d = w.desc()
    inp = make_inputs(w)
    o = OracleRVE(d, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    t = GrainTables(inp["quat"], d["C11"], d["C12"], d["C44"])
    law = _law()
    rho = d["rho0"]
    eps = np.zeros(6)
    epsp = np.zeros(6)
    slipped = False
    for k in range(9):
        de = np.array([0.0, inp["deps"][k], 0, 0, 0, 0])
        st = o.step(de, inp["dt"][k])
        eps = eps + to_mandel2(np.diag([0.0, inp["deps"][k], 0.0])[None])[0]
        g = np.array([d["tau_c0"] + d["mu"] * d["burgers"] * np.sqrt(rho)])
        sig, dg, _, _ = return_map(eps[None], epsp[None], g, inp["dt"][k], t.C, t.S, t.P,
                                   law=law)
        assert np.abs(o.sig - sig).max() <= 1e-9 * np.abs(sig).max()
        assert np.abs(o.rho_gnd).max() <= 1e-6 * rho
        # the committed state: eps_p, rho_SSD from |d beta_p| = |sum dgamma s (x) n|
        dbeta = np.einsum("a,aij->ij", dg[0], t.SN[0])
        epsp = epsp + dg[0] @ t.P[0]
        rho = rho + d["lambda_ssd"] * np.sqrt(2.0 / 3.0 * (dbeta * dbeta).sum())
        slipped |= np.abs(dg).max() > 1e-4
        g_next = d["tau_c0"] + d["mu"] * d["burgers"] * np.sqrt(rho)
        assert np.abs(o.g - g_next).max() <= 1e-9 * g_next
    assert slipped


def test_gnd_coupled_homogeneous_crystal_is_an_implicit_material_point():
    """With the GND coupling the strength of an increment is that of its own end.  For one
    grain the Nye tensor vanishes, so each increment is the material point whose strength
    solves g = tau_c0 + mu b sqrt(rho_SSD,n + lambda sqrt(2/3 |d beta(g)|^2)), d beta(g)
    the slip of the return map at strength g: a scalar root (brentq)."""
    w = small_polycrystal(n=4, n_grains=1, seed=21, cycles=1, incs_per_cycle=20,
                          **cmsx4()).parity()
    d = dict(w.desc(), gnd_coupling=1)
    inp = make_inputs(w)
    o = OracleRVE(d, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    t = GrainTables(inp["quat"], d["C11"], d["C12"], d["C44"])
    law = _law()
    mub = d["mu"] * d["burgers"]
    rho = d["rho0"]
    eps = np.zeros(6)
    epsp = np.zeros(6)
    slipped = 0
    for k in range(9):
        st = o.step(np.array([0.0, inp["deps"][k], 0, 0, 0, 0]), inp["dt"][k])
        eps = eps + to_mandel2(np.diag([0.0, inp["deps"][k], 0.0])[None])[0]

        def slip(g):
            sig, dg, _, _ = return_map(eps[None], epsp[None], np.array([g]), inp["dt"][k], t.C,
                                       t.S, t.P, law=law)
            db = np.einsum("a,aij->ij", dg[0], t.SN[0])
            return sig, dg, rho + d["lambda_ssd"] * np.sqrt(2.0 / 3.0 * (db * db).sum())

        f = lambda g: g - (d["tau_c0"] + mub * np.sqrt(slip(g)[2]))
        g_lo = d["tau_c0"] + mub * np.sqrt(rho)
        if f(g_lo) >= 0.0:                 # no slip: the strength of t_n
            g = g_lo
        else:
            g = brentq(f, g_lo, g_lo + 1e9, xtol=1e-12, rtol=4e-15)
            slipped += 1
            assert st["stag"] >= 2          # the strength moved: at least one more pass
        sig, dg, rho = slip(g)
        epsp = epsp + dg[0] @ t.P[0]
        assert abs(o.g[0] - g) <= 1e-9 * g, (k, o.g[0], g)
        assert np.abs(o.sig[0] - sig[0]).max() <= 1e-8 * np.abs(sig).max()
        assert abs(o.rho_ssd[0] - rho) <= 1e-9 * rho
    assert slipped >= 3


def test_gnd_coupled_polycrystal_is_a_fixed_point():
    """A yielding polycrystal with the GND coupling: after each increment the stress is the
    return map at the committed strain with the committed (end-of-increment) strength, that
    strength is the Taylor strength of the committed SSD and GND densities, the GND density
    is that of the committed plastic distortion, and the coupling changes the answer of the
    lagged reading (non-zero GND hardening within the increment)."""
    from oracle import nye_tensor, gnd_density
    w = small_polycrystal(n=(8, 8, 8), n_grains=3, seed=5, cycles=1, incs_per_cycle=20,
                          **cmsx4()).parity()
    inp = make_inputs(w)
    # the strength fixed point contracts by about 1/2 per alternating pass down to the
    # noise of the inner Newton and Krylov solves (about 1e-11 at their tolerances), so its
    # ratio test runs at 1e-9 (a strength error of ~1e-9 of its change, ~0.02 Pa)
    dc = dict(w.desc(), gnd_coupling=1, tol_stag=1e-9)
    oc = OracleRVE(dc, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ol = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    t = oc.tab
    gid = oc.gid
    mub = dc["mu"] * dc["burgers"]
    for k in range(6):
        de = np.array([0.0, inp["deps"][k], 0, 0, 0, 0])
        epsp_n = to_mandel2(oc.epsp).copy()
        oc.step(de, inp["dt"][k])
        ol.step(de, inp["dt"][k])
        sig, _, _, _ = return_map(to_mandel2(oc.eps), epsp_n, oc.g, inp["dt"][k], t.C[gid],
                                  t.S[gid], t.P[gid], law=_law())
        assert np.abs(sig - oc.sig).max() <= 1e-7 * np.abs(oc.sig).max(), k
        g = dc["tau_c0"] + mub * np.sqrt(oc.rho_ssd + oc.rho_gnd)
        assert np.abs(oc.g - g).max() <= 1e-12 * g.max()
        rg = gnd_density(nye_tensor(oc.grid, oc.beta, dc["ell_fp"]), t.R[gid], dc["burgers"])
        assert np.abs(oc.rho_gnd - rg).max() <= 1e-9 * max(rg.max(), 1.0)
    assert oc.rho_gnd.max() > 1e-3 * oc.rho_ssd.max()
    assert np.abs(oc.g - ol.g).max() > 1e-6 * oc.g.max()


def test_gnd_coupled_relaxation_reaches_the_plain_iterations_fixed_point():
    """The coupled strength is resolved with Aitken's delta-squared relaxation of the
    fixed point g = T(g) (Irons and Tuck); the fixed point does not depend on how it is
    reached: where the plain alternating iteration converges, the relaxed one reaches the
    same strength, stress and strain, in no more passes."""
    w = small_polycrystal(n=(8, 8, 8), n_grains=3, seed=5, cycles=1, incs_per_cycle=20,
                          **cmsx4()).parity()
    inp = make_inputs(w)
    base = dict(w.desc(), gnd_coupling=1, tol_stag=1e-9)
    orx = OracleRVE(base, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    opl = OracleRVE(dict(base, gnd_relax=0), inp["grain"], inp["quat"], inp["tau_c0"],
                    inp["phi0"])
    assert orx.relax and not opl.relax
    passes = [0, 0]
    for k in range(4):
        de = np.array([0.0, inp["deps"][k], 0, 0, 0, 0])
        sr = orx.step(de, inp["dt"][k])
        sp = opl.step(de, inp["dt"][k])
        passes[0] += sr["stag"]
        passes[1] += sp["stag"]
        assert np.abs(orx.g - opl.g).max() <= 1e-7 * np.abs(opl.g - opl.tau0).max(), k
        assert np.abs(orx.sig - opl.sig).max() <= 1e-7 * np.abs(opl.sig).max(), k
        assert np.abs(orx.eps - opl.eps).max() <= 1e-7 * np.abs(opl.eps).max(), k
    assert passes[0] <= passes[1], passes
