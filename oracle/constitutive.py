"""Per-voxel crystal plasticity for the oracle (test infrastructure).

Small-strain form of Sec. 2.1: plastic strain rate = sum of slip rates times
the symmetric Schmid tensors P_a = sym(s_a (x) n_a) (eq. for L_p), tau_a =
P_a : sigma.  Two flow rules give the slip increment over a step dt:

* power law (the paper allows any constitutive choice):
      dgamma_a = dt gdot0 sign(tau_a) |tau_a / g|^n;
* thermally activated glide (eq. flowrule), with A = rho_m b^2 v_D exp(-dF / kT)
  and beta = dV / kT:
      dgamma_a = dt A sign(tau_a) sinh(beta <|tau_a| - g>),   <x> = max(x, 0),
  read as no slip below the critical resolved shear stress g and slip in the
  direction of tau_a (the printed form is the magnitude above the threshold).

Backward Euler on the stress with the slip resistance g frozen at the start of the
increment:

    R(sigma) = C^-1 : (sigma - sigma_tr) + sum_a dgamma_a(tau_a) P_a = 0,
    sigma_tr = C : (eps - eps_p_n).

R is the gradient of the strictly convex potential
    Phi(sigma) = 1/2 (sigma - sigma_tr) : C^-1 : (sigma - sigma_tr) + sum_a phi_a(tau_a),
    phi_a = dt gdot0 g / (n+1) |tau_a / g|^(n+1)                 (power law),
    phi_a = dt A / beta (cosh(beta <|tau_a| - g>) - 1)           (thermally activated),
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


class PowerLaw:
    """dgamma = dt gdot0 sign(tau) |tau/g|^n."""

    def __init__(self, gdot0, n_exp):
        self.gdot0, self.n_exp = float(gdot0), float(n_exp)

    def increments(self, tau, g, dt):
        return slip_increments(tau, g, dt, self.gdot0, self.n_exp)

    def potential(self, tau, g, dt):
        """sum_a dt gdot0 g/(n+1) |tau_a/g|^(n+1), written as |tau| |tau/g|^n so that
        g = inf (no slip) gives 0."""
        n = self.n_exp
        return dt * self.gdot0 / (n + 1.0) * (np.abs(tau) * np.abs(tau / g[:, None]) ** n).sum(1)


class DunneLaw:
    """Thermally activated glide over obstacles (eq. flowrule):
    dgamma = dt A sign(tau) sinh(beta <|tau| - g>), A = rho_m b^2 v_D exp(-dF/(k T)),
    beta = dV/(k T); g is the critical resolved shear stress."""

    def __init__(self, rho_m, burgers, v_D, dF, k_B, T, dV):
        kT = k_B * T
        self.A = rho_m * burgers ** 2 * v_D * np.exp(-dF / kT)
        self.beta = dV / kT

    def _over(self, tau, g):
        # beta <|tau| - g>; g = inf gives 0
        return self.beta * np.maximum(np.abs(tau) - g[..., None], 0.0)

    def increments(self, tau, g, dt):
        with np.errstate(over="ignore", invalid="ignore"):
            x = self._over(tau, g)
            dgam = dt * self.A * np.sign(tau) * np.sinh(x)
            ddg = np.where(x > 0.0, dt * self.A * self.beta * np.cosh(x), 0.0)
        return dgam, ddg

    def potential(self, tau, g, dt):
        """sum_a dt A/beta (cosh(beta <|tau_a| - g>) - 1), the -1 taken as
        cosh(x) - 1 = 2 sinh(x/2)^2 (no cancellation near the threshold)."""
        with np.errstate(over="ignore"):
            x = self._over(tau, g)
            return (dt * self.A / self.beta * 2.0 * np.sinh(0.5 * x) ** 2).sum(1)


def flow_law(d):
    """Flow rule of a description dict: power law unless d["material"] == 1."""
    if int(d.get("material", 0)) == 1:
        return DunneLaw(d["rho_m"], d["burgers"], d["v_D"], d["dF"], d["k_B"], d["T"], d["dV"])
    return PowerLaw(d["gdot0"], d["n_exp"])


def _potential(sig, sig_tr, S, P, g, dt, law):
    d = sig - sig_tr
    el = 0.5 * np.einsum("mi,mij,mj->m", d, S, d)
    tau = np.einsum("mai,mi->ma", P, sig)
    return el + law.potential(tau, g, dt)


def _residual(sig, sig_tr, S, P, g, dt, law):
    tau = np.einsum("mai,mi->ma", P, sig)
    dgam, ddg = law.increments(tau, g, dt)
    R = np.einsum("mij,mj->mi", S, sig - sig_tr) + np.einsum("ma,mai->mi", dgam, P)
    return R, dgam, ddg


def return_map(eps, epsp, g, dt, C, S, P, gdot0=None, n_exp=None, sig0=None, rtol=1e-13,
               maxit=400, law=None):
    """Stress, slip increments and consistent tangent at total strain ``eps``.

    eps, epsp: (M,6) Mandel; g: (M,); C, S: (M,6,6); P: (M,12,6).
    law: PowerLaw or DunneLaw; by default the power law of (gdot0, n_exp).
    sig0: optional starting stress (M,6), used where its potential does not exceed
    that of the default start, the trial stress scaled down until no |tau_a| exceeds
    g.  The root does not depend on the start.
    Returns sig (M,6), dgam (M,12), K (M,6,6) and the incremental energy w (M,).
    """
    if law is None:
        law = PowerLaw(gdot0, n_exp)
    M = len(eps)
    sig_tr = np.einsum("mij,mj->mi", C, eps - epsp)
    tau_tr = np.einsum("mai,mi->ma", P, sig_tr)
    ratio = np.abs(tau_tr).max(1) / g
    sig = sig_tr * np.minimum(1.0, 1.0 / np.maximum(ratio, 1e-300))[:, None]
    if sig0 is not None:
        # start from whichever of sig0 and the scaled trial stress has the lower
        # potential: far above the threshold of an exponential rule the Newton steps
        # shrink to the rule's stress scale (or the potential overflows)
        s0 = np.array(sig0, dtype=np.float64, copy=True)
        with np.errstate(over="ignore", invalid="ignore"):
            p0 = _potential(s0, sig_tr, S, P, g, dt, law)
            pd = _potential(sig, sig_tr, S, P, g, dt, law)
        ok = np.isfinite(p0) & (p0 <= pd)
        sig[ok] = s0[ok]
    scale = np.abs(sig_tr).max(1) + g
    active = np.ones(M, dtype=bool)
    for _ in range(maxit):
        idx = np.nonzero(active)[0]
        if len(idx) == 0:
            break
        a = (sig[idx], sig_tr[idx], S[idx], P[idx], g[idx], dt, law)
        R, dgam, ddg = _residual(*a)
        J = S[idx] + np.einsum("ma,mai,maj->mij", ddg, P[idx], P[idx])
        d = -np.linalg.solve(J, R[..., None])[..., 0]
        phi0 = _potential(*a)
        slope = np.einsum("mi,mi->m", R, d)
        t = np.ones(len(idx))
        todo = np.ones(len(idx), dtype=bool)
        for _ls in range(60):
            cand = sig[idx] + t[:, None] * d
            phi1 = _potential(cand, *a[1:])          # inf past an overflow: halve again
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
    R, dgam, ddg = _residual(sig, sig_tr, S, P, g, dt, law)
    J = S + np.einsum("ma,mai,maj->mij", ddg, P, P)
    sig = sig - np.linalg.solve(J, R[..., None])[..., 0]
    tau = np.einsum("mai,mi->ma", P, sig)
    dgam, ddg = law.increments(tau, g, dt)
    J = S + np.einsum("ma,mai,maj->mij", ddg, P, P)
    K = np.linalg.inv(J)
    K = 0.5 * (K + np.swapaxes(K, 1, 2))
    # incremental (condensed) energy, whose strain gradient is sig:
    #   w(eps) = 1/2 sig_tr : C^-1 : sig_tr - Phi(sig)
    w = 0.5 * np.einsum("mi,mij,mj->m", sig_tr, S, sig_tr) - _potential(
        sig, sig_tr, S, P, g, dt, law)
    return sig, dgam, K, w
