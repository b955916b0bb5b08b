"""Pins of the oracle's crystal tables and return map (Sec. 2.1, small-strain power-law form)."""
import numpy as np
from scipy.optimize import brentq

from oracle import (GrainTables, return_map, slip_increments, quat_to_rot, cubic_stiffness,
                    rotate4, fcc_slip_systems, to_mandel2, from_mandel2, to_mandel4)
from synth import shoemake_quaternions

C11, C12, C44 = 168.4e9, 121.4e9, 75.4e9
GD0, NEXP = 1e-3, 20.0


def test_slip_systems_are_fcc():
    s, n = fcc_slip_systems()
    assert np.allclose(np.linalg.norm(s, axis=1), 1) and np.allclose(np.linalg.norm(n, axis=1), 1)
    assert np.abs((s * n).sum(1)).max() < 1e-15
    # 4 distinct planes x 3 directions, all <110> / {111}
    assert len({tuple(np.round(np.abs(v) * np.sqrt(3), 6)) for v in n}) == 1
    assert sorted(np.round(np.abs(s[0]) * np.sqrt(2), 6)) == [0, 1, 1]
    dyads = {tuple(np.round(np.outer(a, b).ravel(), 9)) for a, b in zip(s, n)}
    assert len(dyads) == 12


def test_rotation_and_cubic_symmetry():
    q = shoemake_quaternions(5, np.random.default_rng(0))
    R = quat_to_rot(q)
    assert np.allclose(np.einsum("gij,gkj->gik", R, R), np.eye(3), atol=1e-15)
    assert np.allclose(np.linalg.det(R), 1.0)
    C = cubic_stiffness(C11, C12, C44)
    # a 90 degree turn about a cube axis leaves cubic elasticity unchanged
    Rz = np.array([[0.0, -1, 0], [1, 0, 0], [0, 0, 1]])
    assert np.allclose(rotate4(C, Rz), C, rtol=0, atol=1e-3)
    # isotropic special case: lambda delta delta + 2 mu I
    lam, mu = 1.0, 2.0
    Ci = to_mandel4(cubic_stiffness(lam + 2 * mu, lam, mu))
    exact = lam * np.outer([1, 1, 1, 0, 0, 0], [1, 1, 1, 0, 0, 0]) + 2 * mu * np.eye(6)
    assert np.allclose(Ci, exact, atol=1e-14)
    # Mandel round trip preserves double contractions
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, 3)); a = a + a.T
    b = rng.standard_normal((3, 3)); b = b + b.T
    assert np.isclose(to_mandel2(a) @ to_mandel2(b), (a * b).sum())
    assert np.allclose(from_mandel2(to_mandel2(a)), a)


def _one(quat, g=50e6):
    t = GrainTables(quat, C11, C12, C44)
    return t, np.array([g])


def test_elastic_limit():
    t, _ = _one(shoemake_quaternions(1, np.random.default_rng(4)))
    eps = to_mandel2(np.array([[[2e-3, 1e-4, 0], [1e-4, -1e-3, 3e-4], [0, 3e-4, 5e-4]]]))
    sig, dg, K, w = return_map(eps, np.zeros((1, 6)), np.array([1e30]), 1.0, t.C, t.S, t.P,
                               GD0, NEXP)
    ref = np.einsum("ijkl,kl->ij", t.C4[0], from_mandel2(eps)[0])
    assert np.allclose(from_mandel2(sig)[0], ref, rtol=1e-13, atol=0)
    assert np.allclose(K[0], t.C[0], rtol=1e-12)
    # infinite strength: exactly elastic
    sig2, dg2, K2, _ = return_map(eps, np.zeros((1, 6)), np.array([np.inf]), 1.0, t.C, t.S,
                                  t.P, GD0, NEXP)
    assert np.all(dg2 == 0) and np.allclose(K2[0], t.C[0], rtol=1e-14)


def _plastic_case(seed=5):
    t, g = _one(shoemake_quaternions(1, np.random.default_rng(seed)))
    eps = to_mandel2(np.array([[[0.0, 0, 0], [0, 4e-3, 0], [0, 0, -1e-3]]]))
    return t, g, eps


def test_residual_is_zero_in_tensor_form():
    t, g, eps = _plastic_case()
    sig, dg, K, w = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)
    S = from_mandel2(sig)[0]
    tau = np.einsum("aij,ij->a", t.SN[0], S)              # P_a : sigma with s (x) n
    dgam = GD0 * np.sign(tau) * np.abs(tau / g[0]) ** NEXP
    assert np.allclose(dgam, dg[0], rtol=1e-12)
    depsp = np.einsum("a,aij->ij", dgam, 0.5 * (t.SN[0] + np.swapaxes(t.SN[0], 1, 2)))
    sig_ref = np.einsum("ijkl,kl->ij", t.C4[0], from_mandel2(eps)[0] - depsp)
    assert np.abs(sig_ref - S).max() <= 1e-12 * np.abs(S).max()
    assert np.abs(dgam).max() > 1e-4                       # genuinely plastic


def test_unique_root_independent_of_start():
    t, g, eps = _plastic_case()
    a = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)[0]
    start = np.einsum("mij,mj->mi", t.C, eps) * 3.0        # far overshoot
    b = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP, sig0=start)[0]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_tangent_and_energy_against_finite_differences():
    t, g, eps = _plastic_case(7)
    e0 = eps[0]
    sig, _, K, w = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)
    h = 1e-9
    Kfd = np.zeros((6, 6))
    gfd = np.zeros(6)
    for b in range(6):
        ep = e0.copy(); ep[b] += h
        em = e0.copy(); em[b] -= h
        sp, _, _, wp = return_map(ep[None], np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)
        sm, _, _, wm = return_map(em[None], np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)
        Kfd[:, b] = (sp[0] - sm[0]) / (2 * h)
        gfd[b] = (wp[0] - wm[0]) / (2 * h)
    assert np.abs(Kfd - K[0]).max() <= 1e-6 * np.abs(K[0]).max()
    assert np.abs(gfd - sig[0]).max() <= 1e-6 * np.abs(sig[0]).max()
    assert np.all(np.linalg.eigvalsh(K[0]) > 0)


def test_single_slip_system_reduces_to_scalar_equation():
    t, g = _one(shoemake_quaternions(1, np.random.default_rng(9)))
    P1 = t.P[:, :1, :]                                    # keep one system
    eps = to_mandel2(np.array([[[1e-3, 2e-3, 0], [2e-3, 0, 1e-3], [0, 1e-3, -5e-4]]]))
    sig, dg, K, w = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, P1, GD0, NEXP)
    p = P1[0, 0]
    tau_tr = p @ t.C[0] @ eps[0]
    pcp = p @ t.C[0] @ p
    f = lambda tau: tau + pcp * GD0 * np.sign(tau) * abs(tau / g[0]) ** NEXP - tau_tr
    tau = brentq(f, 0.0, tau_tr, xtol=1e-16 * abs(tau_tr), rtol=1e-15, maxiter=500)
    assert abs(p @ sig[0] - tau) <= 1e-12 * abs(tau)
    assert abs(tau_tr) > 2 * g[0]


def test_slip_set_permutation_and_sign_invariance():
    t, g, eps = _plastic_case(11)
    a = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, GD0, NEXP)
    perm = np.random.default_rng(0).permutation(12)
    # flipping s -> -s leaves sym(s (x) n) with the opposite sign; slip then flips sign too
    Pf = t.P[:, perm, :] * np.where(np.arange(12) % 2 == 0, -1.0, 1.0)[None, :, None]
    b = return_map(eps, np.zeros((1, 6)), g, 1.0, t.C, t.S, Pf, GD0, NEXP)
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * np.abs(a[0]).max()
    assert np.abs(a[2] - b[2]).max() <= 1e-11 * np.abs(a[2]).max()


def test_power_law_rate_sensitivity():
    tau = np.array([[50e6, -100e6, 25e6]])
    dg, ddg = slip_increments(tau, np.array([50e6]), 2.0, GD0, NEXP)
    assert np.allclose(dg, 2.0 * GD0 * np.array([[1, -2 ** 20, 0.5 ** 20]]))
    assert np.allclose(ddg, 2.0 * GD0 * NEXP / 50e6 * np.array([[1, 2 ** 19, 0.5 ** 19]]))
