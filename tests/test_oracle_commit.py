"""Pins of the oracle's history commit and tensile elastic energy against closed forms.

Every expected value here is formed from quantities a material point exposes (its strain and
its effective stress) through formulas written out in this file, never from the oracle's own
slip increments or energies:

* eq. decMiehe, read as the strain energy density 1/2 eps+ : C : eps+.  For an isotropic
  stiffness (Lame lambda, mu) it is 1/2 lambda (sum <e_i>+)^2 + mu sum <e_i>+^2 over the
  principal elastic strains e_i, taken here from the trigonometric solution of the
  characteristic cubic;
* eq. tot, the plastic work W_p = sum sigma_{n+1} : d eps_p, with the plastic strain
  increment recovered from the stress as d eps_p = d eps - C^-1 : d sigma (backward Euler
  with the end-of-increment stress, the rectangle rule);
* the stored energy density of Sec. 2.3, G_s = xi sum sigma : d eps_p / sqrt(rho_SSD +
  rho_GND), with the SSD density held at rho_0 (lambda = 0) and a prescribed GND density;
* eq. crit: the history H = max over time of W_e+, the trigger at the first commit with
  G_s >= G_crit, and the threshold W_crit = H + W_p frozen at that commit.

The material point is a one-voxel crystal (every field uniform) with an isotropic cubic
stiffness (C44 = (C11 - C12)/2), so the slip stays crystallographic while the elastic
closed forms hold.
"""
import dataclasses

import numpy as np

from oracle import OracleRVE
from oracle.phasefield import we_plus
from synth import single_crystal, make_inputs

C11, C12 = 168.4e9, 121.4e9
LAM, MU = C12, 0.5 * (C11 - C12)
T6 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def _full(v):
    T = np.zeros((3, 3))
    for a, (i, j) in enumerate(T6):
        T[i, j] = T[j, i] = v[a]
    return T


def _iso_c4():
    d = np.eye(3)
    return (LAM * np.einsum("ij,kl->ijkl", d, d)
            + MU * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def _eigvals_sym3(A):
    """Eigenvalues of a symmetric 3x3 matrix from the characteristic cubic (trigonometric
    form: A = q I + p B with det B = 2 cos(3 theta))."""
    q = np.trace(A) / 3.0
    off = A[0, 1] ** 2 + A[0, 2] ** 2 + A[1, 2] ** 2
    p2 = (A[0, 0] - q) ** 2 + (A[1, 1] - q) ** 2 + (A[2, 2] - q) ** 2 + 2.0 * off
    if p2 == 0.0:
        return np.array([q, q, q])
    p = np.sqrt(p2 / 6.0)
    B = (A - q * np.eye(3)) / p
    r = np.clip(np.linalg.det(B) / 2.0, -1.0, 1.0)
    th = np.arccos(r) / 3.0
    e1 = q + 2.0 * p * np.cos(th)
    e3 = q + 2.0 * p * np.cos(th + 2.0 * np.pi / 3.0)
    return np.array([e1, 3.0 * q - e1 - e3, e3])


def _we_plus_iso(E):
    e = np.maximum(_eigvals_sym3(E), 0.0)
    return 0.5 * LAM * e.sum() ** 2 + MU * (e ** 2).sum()


def _compliance_iso(S):
    """Isotropic elastic strain of a stress tensor: (S - lambda/(3 lambda + 2 mu) tr S I)/(2 mu)."""
    return (S - LAM / (3.0 * LAM + 2.0 * MU) * np.trace(S) * np.eye(3)) / (2.0 * MU)


def test_tensile_energy_closed_forms():
    C4 = _iso_c4()[None]
    for eps in (1e-3, 4e-3):
        uni = np.zeros((1, 3, 3))
        uni[0, 1, 1] = eps
        # uniaxial tension: 1/2 (lambda + 2 mu) eps^2; uniaxial and triaxial compression: 0
        assert abs(we_plus(uni, C4)[0] - 0.5 * (LAM + 2 * MU) * eps ** 2) <= \
            1e-13 * (LAM + 2 * MU) * eps ** 2
        assert we_plus(-uni, C4)[0] == 0.0
        assert we_plus(-eps * np.eye(3)[None], C4)[0] == 0.0
        # hydrostatic tension: all of the energy, 9/2 K eps^2 with K = lambda + 2 mu / 3
        K = LAM + 2.0 * MU / 3.0
        assert abs(we_plus(eps * np.eye(3)[None], C4)[0] - 4.5 * K * eps ** 2) <= \
            1e-13 * K * eps ** 2
    rng = np.random.default_rng(4)
    for _ in range(50):
        A = rng.standard_normal((3, 3)) * 2e-3
        E = 0.5 * (A + A.T)
        ref = _we_plus_iso(E)
        assert abs(we_plus(E[None], C4)[0] - ref) <= 1e-12 * max(ref, 1e-300) + 1e-30


def _point(**kw):
    w = dataclasses.replace(single_crystal(n=1, seed=6, notch=False), C11=C11, C12=C12,
                            C44=MU, **kw).parity()
    inp = make_inputs(w)
    r = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    return w, inp, r


def test_history_of_an_elastic_point_is_the_tensile_energy_envelope():
    # no slip: H after each increment is the largest 1/2 (lambda + 2 mu) <eps_yy>+^2 so far
    w, inp, r = _point(tau_c0=1e12, G_crit=1e30)
    eyy, env = 0.0, 0.0
    for de, dt in zip(inp["deps"][:30], inp["dt"][:30]):
        r.step([0, de, 0, 0, 0, 0], dt)
        eyy += de
        env = max(env, 0.5 * (LAM + 2 * MU) * max(eyy, 0.0) ** 2)
        assert abs(r.H[0] - env) <= 1e-12 * 0.5 * (LAM + 2 * MU) * 0.005 ** 2
    # the power law slips a vanishing amount this far below the strength (~1e-74 J/m^3)
    assert abs(r.Wp[0]) < 1e-50 and abs(r.Gs[0]) < 1e-50 and not r.trig[0]
    assert env > 0.0


def _replay(r, inp, n_inc, rho_gnd):
    """Step the point, holding rho_GND at the prescribed value, and return per increment the
    strain and effective stress (3x3) plus the committed W_p, G_s, H, W_crit, trigger."""
    rows = []
    for de, dt in zip(inp["deps"][:n_inc], inp["dt"][:n_inc]):
        r.rho_gnd[:] = rho_gnd
        r.step([0, de, 0, 0, 0, 0], dt)
        f = r.fields()
        rows.append(dict(eps=_full(f["strain"][0]), sig=_full(f["stress_eff"][0]),
                         wp=r.Wp[0], gs=r.Gs[0], h=r.H[0], wcrit=r.Wcrit[0], trig=bool(r.trig[0]),
                         rho_ssd=r.rho_ssd[0]))
    return rows


def _closed_form_series(rows, xi, rho_total, G_crit):
    wp = gs = h = wcrit = 0.0
    trig = False
    eps_prev = np.zeros((3, 3))
    ee_prev = np.zeros((3, 3))
    out = []
    for row in rows:
        ee = _compliance_iso(row["sig"])
        d_ep = (row["eps"] - eps_prev) - (ee - ee_prev)
        dw = float(np.sum(row["sig"] * d_ep))
        wp += dw
        gs += xi * dw / np.sqrt(rho_total)
        h = max(h, _we_plus_iso(ee))
        if not trig and gs >= G_crit:
            trig, wcrit = True, h + wp
        out.append(dict(wp=wp, gs=gs, h=h, wcrit=wcrit, trig=trig))
        eps_prev, ee_prev = row["eps"], ee
    return out


def test_plastic_work_stored_energy_and_trigger_of_a_yielding_point():
    rho0, rho_gnd = 1e12, 3e12
    # find the stored energy of the 12th increment first, then put G_crit half-way between
    # two consecutive values so that the trigger is not decided by rounding
    w, inp, r = _point(lambda_ssd=0.0, G_crit=1e30, rho0=rho0)
    probe = _closed_form_series(_replay(r, inp, 14, rho_gnd), w.xi_store, rho0 + rho_gnd, 1e30)
    gcrit = 0.5 * (probe[10]["gs"] + probe[11]["gs"])
    assert probe[11]["gs"] > probe[10]["gs"] * (1 + 1e-3)
    w, inp, r = _point(lambda_ssd=0.0, G_crit=gcrit, rho0=rho0)
    rows = _replay(r, inp, 24, rho_gnd)
    ref = _closed_form_series(rows, w.xi_store, rho0 + rho_gnd, gcrit)
    wp_scale = max(abs(x["wp"]) for x in ref)
    assert wp_scale > 1e3        # the point yields: several kJ/m^3 of plastic work
    for k, (got, exp) in enumerate(zip(rows, ref)):
        assert abs(got["wp"] - exp["wp"]) <= 1e-8 * wp_scale, (k, got["wp"], exp["wp"])
        assert abs(got["gs"] - exp["gs"]) <= 1e-8 * abs(ref[-1]["gs"]), (k, got["gs"], exp["gs"])
        assert abs(got["h"] - exp["h"]) <= 1e-10 * max(x["h"] for x in ref), k
        assert got["trig"] == exp["trig"], k
        assert abs(got["wcrit"] - exp["wcrit"]) <= 1e-8 * wp_scale, (k, got["wcrit"],
                                                                      exp["wcrit"])
        assert got["rho_ssd"] == rho0
    assert rows[10]["trig"] is False and rows[11]["trig"] is True
    assert ref[11]["wcrit"] > ref[11]["h"] > 0.0 and ref[11]["wp"] > 0.0
    # once triggered, the threshold stays frozen while H and W_p keep growing
    assert all(x["wcrit"] == ref[11]["wcrit"] for x in ref[11:])
    assert ref[-1]["wp"] > ref[11]["wp"]


def test_hardening_ssd_and_stored_energy_under_single_slip():
    """Strain along the Schmid tensor P = sym(s (x) n) of one FCC system (s = [1,-1,0]/sqrt2,
    n = [1,1,1]/sqrt3, identity orientation) with an isotropic stiffness: the stress stays
    along P, the resolved stress of every other system is at most 2/3 of this one's, and at
    a rate exponent of 60 their slip is ~(2/3)^60 ~ 3e-11 of it.  Then d eps_p = dgamma P,
    so |dgamma| = sqrt2 |d eps_p|, and Sec. 2.1 gives in closed form
        g       += h_lin |dgamma|,
        rho_SSD += lambda sqrt(2/3 dLp : dLp) = lambda sqrt(2/3) |dgamma|   (dLp = dgamma s (x) n),
        G_s     += xi sigma : d eps_p / sqrt(rho_SSD,n+1 + rho_GND)."""
    s = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    n = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    P = 0.5 * (np.outer(s, n) + np.outer(n, s))
    p6 = np.array([P[i, j] for (i, j) in T6])
    w = dataclasses.replace(single_crystal(n=1, seed=6, notch=False), C11=C11, C12=C12, C44=MU,
                            n_exp=60.0, G_crit=1e30).parity()
    d = w.desc()
    r = OracleRVE(d, np.zeros(1, dtype=np.int32), np.array([[1.0, 0.0, 0.0, 0.0]]))
    inp = make_inputs(w)
    rho_gnd = 2e12
    g_ref, rho_ref, gs_ref, wp_ref = d["tau_c0"], d["rho0"], 0.0, 0.0
    eps_prev = ee_prev = np.zeros((3, 3))
    slipped = 0
    for k in range(20):
        de, dt = 4.0 * inp["deps"][k], inp["dt"][k]
        r.rho_gnd[:] = rho_gnd
        r.step(list(de * p6), dt)
        f = r.fields()
        eps, sig = _full(f["strain"][0]), _full(f["stress_eff"][0])
        ee = _compliance_iso(sig)
        d_ep = (eps - eps_prev) - (ee - ee_prev)
        dgam = np.sqrt(2.0) * np.linalg.norm(d_ep)
        # the plastic strain increment is along P (single slip) to the stated accuracy
        # (above a 1e-15 floor: the rounding of a strain recovered from a stress)
        assert np.linalg.norm(d_ep - np.sum(d_ep * P) / np.sum(P * P) * P) <= \
            1e-9 * np.linalg.norm(d_ep) + 1e-15
        g_ref += d["h_lin"] * dgam
        rho_ref += d["lambda_ssd"] * np.sqrt(2.0 / 3.0) * dgam
        dw = float(np.sum(sig * d_ep))
        wp_ref += dw
        gs_ref += d["xi_store"] * dw / np.sqrt(rho_ref + rho_gnd)
        assert abs(f["g"][0] - g_ref) <= 1e-9 * g_ref, (k, f["g"][0], g_ref)
        assert abs(r.rho_ssd[0] - rho_ref) <= 1e-9 * rho_ref, (k, r.rho_ssd[0], rho_ref)
        assert abs(r.Wp[0] - wp_ref) <= 1e-8 * max(abs(wp_ref), 1.0), (k, r.Wp[0], wp_ref)
        assert abs(r.Gs[0] - gs_ref) <= 1e-8 * max(abs(gs_ref), 1e-12), (k, r.Gs[0], gs_ref)
        slipped += dgam > 1e-5
        eps_prev, ee_prev = eps, ee
    assert slipped >= 5 and g_ref > 1.2 * d["tau_c0"] and rho_ref > 1.5 * d["rho0"]
