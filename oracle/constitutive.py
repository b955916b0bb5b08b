"""Per-voxel crystal plasticity for the oracle (test infrastructure).

Small-strain form of Sec. 2.1: plastic strain rate = sum of slip rates times
the symmetric Schmid tensors P_a = sym(s_a (x) n_a) (eq. for L_p).  Flow rule:
power law  dgamma_a = dt * gdot0 * sign(tau_a) * |tau_a / g|^n  with tau_a =
P_a : sigma (the paper allows any constitutive choice).  Backward Euler on the
stress with the slip resistance g frozen at the start of the increment:

    R(sigma) = C^-1 : (sigma - sigma_tr) + sum_a dgamma_a(tau_a) P_a = 0,
    sigma_tr = C : (eps - eps_p_n).

R is the gradient of the strictly convex potential
    Phi(sigma) = 1/2 (sigma - sigma_tr) : C^-1 : (sigma - sigma_tr)
                 + sum_a dt gdot0 g / (n+1) |tau_a / g|^(n+1),
so the root is unique; it is found by Newton's method with backtracking on
Phi.  A voxel with g = inf never slips (linear elastic).  The consistent tangent (needed by eq. newton) is
    K = d sigma / d eps = (C^-1 + sum_a d(dgamma_a)/d tau_a  P_a (x) P_a)^-1.
The incremental energy w(eps) = 1/2 sig_tr : C^-1 : sig_tr - Phi(sig*) is convex in
eps with gradient sig and Hessian K, which gives the momentum Newton solver a
merit function.  Everything is in Mandel 6-vector / 6x6 form.
"""
import numpy as np

from .crystal import (quat_to_rot, cubic_stiffness, rotate4, fcc_slip_systems, to_mandel2,
                      to_mandel4)


class GrainTables:
    """Per-grain rotated stiffness, compliance and Schmid tensors (sample frame)."""

    def __init__(self, quat, C11, C12, C44):
        R = quat_to_rot(np.atleast_2d(quat))
        self.R = R
        C0 = cubic_stiffness(C11, C12, C44)
        s0, n0 = fcc_slip_systems()
        G = len(R)
        self.C4 = np.array([rotate4(C0, R[g]) for g in range(G)])
        self.C = to_mandel4(self.C4)
        self.S = np.linalg.inv(self.C)
        s = np.einsum("gij,aj->gai", R, s0)
        n = np.einsum("gij,aj->gai", R, n0)
        self.s = s
        self.n = n
        self.SN = np.einsum("gai,gaj->gaij", s, n)            # s (x) n, (G,12,3,3)
        self.P = to_mandel2(self.SN)                          # Mandel of sym(s (x) n)


def slip_increments(tau, g, dt, gdot0, n_exp):
    """Power-law slip increments and their derivatives d(dgamma)/d(tau)."""
    x = tau / g[..., None]
    ax = np.abs(x)
    dgam = dt * gdot0 * np.sign(x) * ax ** n_exp
    ddg = dt * gdot0 * n_exp / g[..., None] * ax ** (n_exp - 1.0)
    return dgam, ddg


def _potential(sig, sig_tr, S, P, g, dt, gdot0, n_exp):
    d = sig - sig_tr
    el = 0.5 * np.einsum("mi,mij,mj->m", d, S, d)
    tau = np.einsum("mai,mi->ma", P, sig)
    # g |tau/g|^(n+1) written as |tau| |tau/g|^n so that g = inf (no slip) gives 0
    pl = dt * gdot0 / (n_exp + 1.0) * (np.abs(tau) * np.abs(tau / g[:, None]) ** n_exp).sum(1)
    return el + pl


def _residual(sig, sig_tr, S, P, g, dt, gdot0, n_exp):
    tau = np.einsum("mai,mi->ma", P, sig)
    dgam, ddg = slip_increments(tau, g, dt, gdot0, n_exp)
    R = np.einsum("mij,mj->mi", S, sig - sig_tr) + np.einsum("ma,mai->mi", dgam, P)
    return R, dgam, ddg


def return_map(eps, epsp, g, dt, C, S, P, gdot0, n_exp, sig0=None, rtol=1e-13, maxit=400):
    """Stress, slip increments and consistent tangent at total strain ``eps``.

    eps, epsp: (M,6) Mandel; g: (M,); C, S: (M,6,6); P: (M,12,6).
    sig0: optional starting stress (M,6); the default is the trial stress scaled
    down until no |tau_a| exceeds g.  The root does not depend on the start.
    Returns sig (M,6), dgam (M,12), K (M,6,6) and the incremental energy w (M,).
    """
    M = len(eps)
    sig_tr = np.einsum("mij,mj->mi", C, eps - epsp)
    if sig0 is None:
        tau_tr = np.einsum("mai,mi->ma", P, sig_tr)
        ratio = np.abs(tau_tr).max(1) / g
        sig = sig_tr * np.minimum(1.0, 1.0 / np.maximum(ratio, 1e-300))[:, None]
    else:
        sig = np.array(sig0, dtype=np.float64, copy=True)
    scale = np.abs(sig_tr).max(1) + g
    active = np.ones(M, dtype=bool)
    for _ in range(maxit):
        idx = np.nonzero(active)[0]
        if len(idx) == 0:
            break
        a = (sig[idx], sig_tr[idx], S[idx], P[idx], g[idx], dt, gdot0, n_exp)
        R, dgam, ddg = _residual(*a)
        J = S[idx] + np.einsum("ma,mai,maj->mij", ddg, P[idx], P[idx])
        d = -np.linalg.solve(J, R[..., None])[..., 0]
        phi0 = _potential(*a)
        slope = np.einsum("mi,mi->m", R, d)
        t = np.ones(len(idx))
        todo = np.ones(len(idx), dtype=bool)
        for _ls in range(60):
            cand = sig[idx] + t[:, None] * d
            phi1 = _potential(cand, *a[1:])
            ok = phi1 <= phi0 + 1e-4 * t * slope + 1e-13 * np.abs(phi0)
            todo &= ~ok
            if not todo.any():
                break
            t = np.where(todo, 0.5 * t, t)
        step = t[:, None] * d
        sig[idx] = sig[idx] + step
        small = np.abs(step).max(1) <= rtol * scale[idx]
        active[idx[small]] = False
    if active.any():
        raise RuntimeError(f"return map did not converge at {active.sum()} voxels")
    # polish once more and evaluate the tangent at the root
    R, dgam, ddg = _residual(sig, sig_tr, S, P, g, dt, gdot0, n_exp)
    J = S + np.einsum("ma,mai,maj->mij", ddg, P, P)
    sig = sig - np.linalg.solve(J, R[..., None])[..., 0]
    tau = np.einsum("mai,mi->ma", P, sig)
    dgam, ddg = slip_increments(tau, g, dt, gdot0, n_exp)
    J = S + np.einsum("ma,mai,maj->mij", ddg, P, P)
    K = np.linalg.inv(J)
    K = 0.5 * (K + np.swapaxes(K, 1, 2))
    # incremental (condensed) energy, whose strain gradient is sig:
    #   w(eps) = 1/2 sig_tr : C^-1 : sig_tr - Phi(sig)
    w = 0.5 * np.einsum("mi,mij,mj->m", sig_tr, S, sig_tr) - _potential(
        sig, sig_tr, S, P, g, dt, gdot0, n_exp)
    return sig, dgam, K, w
