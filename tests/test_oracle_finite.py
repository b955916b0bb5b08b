"""Pins of the finite-strain oracle (Sec. 2.1 kinematics, Sec. 3.1 eqs. fdef and newton,
eq. decMiehe with the logarithmic elastic strain) against what the mechanics fixes:

* a rigid rotation is stress free, and the update is objective: P(Q F) = Q P(F) with the
  same plastic deformation and slip;
* the small-strain limit: at F = I + delta E the first Piola-Kirchhoff stress tends to the
  small-strain oracle's stress at eps = delta sym(E) (elastic and yielding), the relative
  difference shrinking linearly with delta;
* the consistent tangent equals central differences of P(F);
* the log-strain tensile energy of an isotropic lattice in closed form (Hencky), for any
  elastic rotation;
* the increment solver: a homogeneous crystal stays homogeneous (a material point), and a
  yielding polycrystal's converged state is equilibrated (zero Fourier divergence of the
  degraded P) and compatible (zero Fourier curl of F - F_bar) at the tight tolerances.
"""
import dataclasses

import numpy as np
import pytest

from oracle import GrainTables, return_map, to_mandel2, from_mandel2, PowerLaw
from oracle.finite import (fs_return_map, fs_tangent, we_plus_log, OracleFiniteRVE, grad_hat)
from synth import single_crystal, small_polycrystal, make_inputs

C11, C12, C44 = 168.4e9, 121.4e9, 75.4e9


def _rot(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0] = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1)
    R[:, 1] = np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1)
    R[:, 2] = np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)
    return R, q


def _setup(M=64, seed=0, g=50e6):
    rng = np.random.default_rng(seed)
    _, q = _rot(rng, 5)
    tab = GrainTables(q, C11, C12, C44)
    gid = rng.integers(0, 5, M)
    return rng, tab, gid, np.full(M, g), PowerLaw(1e-3, 20.0)


def test_rigid_rotation_is_stress_free_and_update_is_objective():
    rng, tab, gid, g, law = _setup()
    M = len(gid)
    Q, _ = _rot(rng, M)
    r = fs_return_map(Q, np.tile(np.eye(3), (M, 1, 1)), g, 1.0, tab, gid, law)
    # zero up to the rounding of Q^T Q - I (1e-16) times the stiffness
    assert np.abs(r["P"]).max() <= 1e-14 * C11 and np.abs(r["dgam"]).max() <= 1e-200
    # a yielding state: stretch + shear with a plastic history
    F = np.eye(3) + rng.uniform(-6e-3, 6e-3, (M, 3, 3))
    Fp = np.eye(3) + rng.uniform(-2e-3, 2e-3, (M, 3, 3))
    a = fs_return_map(F, Fp, g, 1.0, tab, gid, law)
    b = fs_return_map(Q @ F, Fp, g, 1.0, tab, gid, law)
    assert np.abs(a["dgam"]).max() > 1e-4                       # genuinely plastic
    scale = np.abs(a["P"]).max()
    assert np.abs(b["P"] - Q @ a["P"]).max() <= 1e-11 * scale
    assert np.abs(b["Fp_new"] - a["Fp_new"]).max() <= 1e-13
    assert np.abs(b["dgam"] - a["dgam"]).max() <= 1e-12 * np.abs(a["dgam"]).max()


@pytest.mark.parametrize("g", [1e12, 50e6])
def test_small_strain_limit(g):
    rng, tab, gid, gg, law = _setup(g=g)
    M = len(gid)
    E = rng.uniform(-1.0, 1.0, (M, 3, 3))
    E[:, 1, 1] += 1.5
    errs = []
    for delta in (4e-3, 4e-4, 4e-5):
        F = np.eye(3) + delta * E
        r = fs_return_map(F, np.tile(np.eye(3), (M, 1, 1)), gg, 1.0, tab, gid, law)
        eps = to_mandel2(delta * 0.5 * (E + np.swapaxes(E, 1, 2)))
        sig, dg, _, _ = return_map(eps, np.zeros_like(eps), gg, 1.0, tab.C[gid], tab.S[gid],
                                   tab.P[gid], law=law)
        ref = from_mandel2(sig)
        errs.append(np.abs(r["P"] - ref).max() / np.abs(ref).max())
    print("relative |P - sigma|:", errs)
    assert errs[1] <= 0.15 * errs[0] and errs[2] <= 0.15 * errs[1]
    assert errs[2] <= 2e-3


def test_consistent_tangent_matches_central_differences():
    rng, tab, gid, g, law = _setup(M=24, seed=3)
    M = len(gid)
    F = np.eye(3) + rng.uniform(-5e-3, 5e-3, (M, 3, 3))
    F[:, 1, 1] += 4e-3
    Fp = np.eye(3) + rng.uniform(-1e-3, 1e-3, (M, 3, 3))
    r = fs_return_map(F, Fp, g, 1.0, tab, gid, law)
    assert np.abs(r["dgam"]).max() > 1e-4
    K = fs_tangent(F, r)
    h = 1e-7
    Kfd = np.empty_like(K)
    for k in range(3):
        for l in range(3):
            dF = np.zeros((M, 3, 3))
            dF[:, k, l] = h
            Pp = fs_return_map(F + dF, Fp, g, 1.0, tab, gid, law)["P"]
            Pm = fs_return_map(F - dF, Fp, g, 1.0, tab, gid, law)["P"]
            Kfd[:, :, :, k, l] = (Pp - Pm) / (2 * h)
    err = np.abs(K - Kfd).max() / np.abs(K).max()
    print(f"tangent vs central differences: {err:.2e}")
    assert err <= 2e-6
    # and not the small-strain tangent: the rotational part of P matters
    assert np.abs(K - np.swapaxes(K, 1, 2)).max() > 1e-3 * np.abs(K).max()


def test_log_strain_tensile_energy_closed_form():
    lam, mu = C12, 0.5 * (C11 - C12)
    d = np.eye(3)
    C4 = (lam * np.einsum("ij,kl->ijkl", d, d)
          + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    rng = np.random.default_rng(2)
    Q, _ = _rot(rng, 40)
    stretch = np.exp(rng.uniform(-4e-3, 4e-3, (40, 3)))
    Fe = Q @ (stretch[:, :, None] * np.eye(3)[None])              # Fe = Q diag(stretch)
    e = np.maximum(np.log(stretch), 0.0)
    ref = 0.5 * lam * e.sum(1) ** 2 + mu * (e ** 2).sum(1)
    got = we_plus_log(Fe, np.broadcast_to(C4, (40, 3, 3, 3, 3)))
    assert np.abs(got - ref).max() <= 1e-12 * ref.max()
    # also with the stretch axes turned (Fe = Q U with U = V diag V^T): the energy
    # depends only on the principal stretches
    V, _ = _rot(rng, 40)
    U = V @ (stretch[:, :, None] * np.eye(3)[None]) @ np.swapaxes(V, 1, 2)
    got2 = we_plus_log(Q @ U, np.broadcast_to(C4, (40, 3, 3, 3, 3)))
    assert np.abs(got2 - ref).max() <= 1e-12 * ref.max()


def _fs_rve(w):
    inp = make_inputs(w)
    return inp, OracleFiniteRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])


def test_homogeneous_crystal_stays_a_material_point():
    w = single_crystal(n=4, seed=3, notch=False).parity()
    inp, r = _fs_rve(w)
    Fbar = np.eye(3)
    for de, dt in zip(inp["deps"][:6], inp["dt"][:6]):
        dF = np.zeros((3, 3))
        dF[1, 1] = de
        r.step(dF.ravel(), dt)
        Fbar = Fbar + dF
        assert np.abs(r.F - Fbar[None]).max() <= 1e-15
        assert np.ptp(r.P.reshape(-1, 9), axis=0).max() <= 1e-9 * np.abs(r.P).max()
    assert np.abs(r.Wp).max() > 0.0                              # it yielded


def test_polycrystal_increments_are_equilibrated_and_compatible():
    w = dataclasses.replace(small_polycrystal(n=(8, 6, 4), n_grains=3, seed=4),
                            amplitude=0.008).parity()
    inp, r = _fs_rve(w)
    Fbar = np.eye(3)
    for de, dt in zip(inp["deps"][:4], inp["dt"][:4]):
        dF = np.zeros((3, 3))
        dF[1, 1] = de
        st = r.step(dF.ravel(), dt)
        Fbar = Fbar + dF
    g = r.grid
    f = r.fields()
    assert np.abs(f["defgrad"].mean(0) - Fbar.ravel()).max() <= 1e-15
    Ph = g.fft(g.to_grid(f["pk1"].reshape(-1, 3, 3)))
    div = np.abs(g.div_hat(Ph)).max() / (np.abs(Ph).max() * np.abs(g.xit).max())
    # compatibility: F - F_bar = grad u  <=>  its Fourier curl (rows) vanishes
    Fh = g.fft(g.to_grid(f["defgrad"].reshape(-1, 3, 3) - Fbar[None]))
    curl = np.abs(g.curl_hat(Fh)).max() / (np.abs(Fh).max() * np.abs(g.xit).max())
    print(f"equilibrium {div:.2e}, compatibility {curl:.2e}, newton {st['newton']}")
    assert div <= 1e-10 and curl <= 1e-12
    assert np.abs(r.Wp).max() > 0.0 and np.ptp(r.Wp) > 0.0
    # plastic incompressibility to first order: det Fp = 1 + O(dgamma^2)
    dets = np.linalg.det(r.Fp)
    assert np.abs(dets - 1.0).max() <= 1e-4


def _iso_tab():
    lam, mu = C12, 0.5 * (C11 - C12)
    return lam, mu, GrainTables(np.array([[1.0, 0.0, 0.0, 0.0]]), C11, C12, mu)


def test_elastic_first_piola_kirchhoff_is_the_energy_gradient():
    """No slip: P = dW/dF of W = 1/2 Ee : C : Ee, Ee = 1/2 (Fe^T Fe - I), Fe = F Fp^-1,
    per unit reference volume of the intermediate configuration (det Fp = 1 here)."""
    lam, mu, tab = _iso_tab()
    rng = np.random.default_rng(7)
    M = 12
    F = np.eye(3) + rng.uniform(-0.03, 0.03, (M, 3, 3))
    Fp = np.eye(3) + 0.02 * (rng.uniform(-1, 1, (M, 3, 3)))
    Fp /= np.cbrt(np.linalg.det(Fp))[:, None, None]
    gid = np.zeros(M, dtype=np.int64)
    r = fs_return_map(F, Fp, np.full(M, 1e30), 1.0, tab, gid, PowerLaw(1e-3, 20.0))

    def W(F_):
        Fe = F_ @ np.linalg.inv(Fp)
        E = 0.5 * (np.swapaxes(Fe, 1, 2) @ Fe - np.eye(3))
        tr = np.trace(E, axis1=1, axis2=2)
        return 0.5 * lam * tr ** 2 + mu * np.einsum("mij,mij->m", E, E)

    h = 1e-7
    G = np.empty((M, 3, 3))
    for k in range(3):
        for l in range(3):
            dF = np.zeros((M, 3, 3))
            dF[:, k, l] = h
            G[:, k, l] = (W(F + dF) - W(F - dF)) / (2 * h)
    err = np.abs(r["P"] - G).max() / np.abs(G).max()
    print(f"P vs energy gradient: {err:.2e}")
    assert err <= 1e-6


def test_single_slip_reduces_to_a_scalar_root():
    """F = I + gamma s (x) n on one FCC system (identity orientation, isotropic lattice,
    rate exponent 60 so that the other systems, resolved at most 2/3 as high, slip
    (2/3)^60 ~ 3e-11 as much), Fp_n = I + gp s (x) n.  s (x) n is nilpotent, so the
    update's products are exact: Fe* = I + ge s (x) n with ge = gamma - gp,
    A = I + 2 ge P0 + ge^2 n (x) n, and the return map is one equation in dgamma:
        Ee = 1/2 (A - I) - dgamma sym(A s (x) n),  S = lambda tr(Ee) I + 2 mu Ee,
        dgamma = dt gdot0 sign(tau) |tau/g|^60,  tau = S : sym(A s (x) n),
    after which Fp_{n+1}^-1 = I - (gp + dgamma) s (x) n and P = F Fp^-1 S Fp^-T."""
    from scipy.optimize import brentq
    lam, mu, tab = _iso_tab()
    s = np.array([1.0, -1.0, 0.0]) / np.sqrt(2.0)
    n = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    S0 = np.outer(s, n)
    law = PowerLaw(1e-3, 60.0)
    g = 50e6
    for gamma, gp in ((0.004, 0.001), (0.02, 0.012), (-0.01, 0.002)):
        ge = gamma - gp
        A = np.eye(3) + ge * (S0 + S0.T) + ge * ge * np.outer(n, n)
        Q0 = 0.5 * (A @ S0 + (A @ S0).T)

        def stress(dg):
            Ee = 0.5 * (A - np.eye(3)) - dg * Q0
            return lam * np.trace(Ee) * np.eye(3) + 2.0 * mu * Ee

        def f(dg):
            tau = np.sum(stress(dg) * Q0)
            return dg - np.sign(tau) * abs(tau / g) ** 60 * 1e-3

        lo, hi = (0.0, ge) if ge > 0 else (ge, 0.0)
        dg = brentq(f, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
        S_ref = stress(dg)
        Gi = np.eye(3) - (gp + dg) * S0
        F = np.eye(3) + gamma * S0
        P_ref = F @ Gi @ S_ref @ Gi.T
        r = fs_return_map(F[None], (np.eye(3) + gp * S0)[None], np.array([g]), 1.0, tab,
                          np.zeros(1, dtype=np.int64), law)
        eS = np.abs(from_mandel2(r["S"])[0] - S_ref).max() / np.abs(S_ref).max()
        eP = np.abs(r["P"][0] - P_ref).max() / np.abs(P_ref).max()
        print(f"gamma {gamma}: dgamma {dg:.6e}, S {eS:.1e}, P {eP:.1e}")
        assert abs(dg) > 1e-4                      # it slipped
        assert eS <= 1e-9 and eP <= 1e-9
