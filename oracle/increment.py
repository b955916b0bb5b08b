"""One time increment by non-linear alternating minimisation (oracle).

Algorithm 1 of the paper, small-strain form:
    eps_0 = eps_t + d eps_bar (uniform; under mixed control only the strain-controlled
            components move, the stress-controlled ones are unknowns of the momentum
            Newton system with target macro stress = that of t plus the increment),
    phi_0 = phi_t
    repeat  i = 1, 2, ...
        eps_i  = momentum balance by Newton-Krylov at phi_{i-1}, from eps_{i-1}
        phi_i  = phase-field balance at eps_i, then phi_i = max(phi_i, phi_t)
    until  max|eps_i - eps_{i-1}| / max|eps_i - eps_t| <= tol
      and  max|phi_i - phi_{i-1}| / max|phi_i - phi_t| <= tol   (0/0 read as 0)
followed by the history commit of the internal variables:
    eps_p, beta_p += sum dgamma (P_a, s_a (x) n_a)
    g       += h_lin sum |dgamma|                 (linear hardening, power law)
    g        = tau_c0 + mu b sqrt(rho_SSD + rho_GND)   (Taylor hardening, thermally
               activated flow; from the committed densities, GND included)
    rho_SSD += lambda sqrt(2/3 dLp : dLp)          (SSD evolution, Sec. 2.1)
    W_p     += sigma : d eps_p                     (plastic work, eq. tot)
    G_s     += xi sigma : d eps_p / sqrt(rho_SSD + rho_GND)     (stored energy)
    H        = max(H, W_e+)                        (max tensile energy, eq. crit)
    first time G_s >= G_crit: W_crit = H + W_p     (eq. crit)
and the lagged GND density from the committed plastic distortion.
Readings: phi is also capped at 1; the driving state uses the threshold and the
trigger flag of the start of the increment; rho_GND enters G_s one increment
late; the Taylor strength of an increment is that of the densities committed at
the end of the previous one (g frozen over the step, as for the power law).

Option ``gnd_coupling`` (thermally activated flow with Taylor hardening): the strength
of the increment is that of its own end, g_{n+1} = tau_c0 + mu b sqrt(rho_SSD,n+1 +
rho_GND,n+1), with both densities from the increment's slip (the SSD rate and the
regularised Nye tensor of the plastic distortion beta_n + d beta, non-local), resolved
by the alternating minimisation: each pass solves the momentum balance at the current
strength, recomputes the end-of-increment densities and the strength T(g) from its slip,
and the loop also requires max|T(g_i) - g_i| / max|T(g_i) - g_n| <= tol (0/0 read as 0);
G_s then uses rho_GND,n+1.  The next pass's strength is g_i + omega_i (T(g_i) - g_i)
with Aitken's delta-squared factor (Irons and Tuck; omega_0 = 1/2), since the plain
update g_(i+1) = T(g_i) (option gnd_relax = 0) can stall in yielding polycrystals; both
have the same fixed point.

Option ``plane_stress`` (plates one voxel thick, N3 = 1; Sec. 4.1-4.3): the out-of-plane
stress vanishes at every voxel and the out-of-plane strain is a local unknown
(planestress.py); macro control then names in-plane components only.
"""
import numpy as np

from .constitutive import GrainTables, return_map, flow_law
from .crystal import to_mandel2, from_mandel2
from .spectral import Grid
from .mechanics import solve_mechanics
from .planestress import solve_mechanics_plane
from .phasefield import we_plus, solve_phase_field, solve_phase_field_dirichlet
from .history import nye_tensor, gnd_density

T6 = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def tensor6(T):
    """(M,3,3) -> (M,6) tensor components xx, yy, zz, yz, xz, xy."""
    return np.stack([T[:, i, j] for (i, j) in T6], axis=1)


def from_tensor6(v):
    v = np.atleast_2d(v)
    T = np.empty((len(v), 3, 3))
    for a, (i, j) in enumerate(T6):
        T[:, i, j] = v[:, a]
        T[:, j, i] = v[:, a]
    return T


def _ratio(num, den):
    if num == 0.0:
        return 0.0
    return num / den if den > 0.0 else np.inf


class OracleRVE:
    """State and increments of one periodic RVE.  ``desc`` is a flat dict of constants
    (see ``synth.Workload.desc``); arrays are flat with x fastest."""

    def __init__(self, desc, grain, quat, tau_c0=None, phi0=None):
        self.d = dict(desc)
        d = self.d
        self.grid = Grid(d["n"], d["h"], d.get("scheme", 0))
        M = self.grid.M
        self.gid = np.asarray(grain, dtype=np.int64)
        quat = np.atleast_2d(np.asarray(quat, dtype=np.float64))
        self.tab = GrainTables(quat, d["C11"], d["C12"], d["C44"])
        G = len(quat)
        tau = np.full(G, d["tau_c0"]) if tau_c0 is None else np.asarray(tau_c0, dtype=float)
        self.eps = np.zeros((M, 3, 3))
        self.epsp = np.zeros((M, 3, 3))
        self.beta = np.zeros((M, 3, 3))
        self.law = flow_law(d)
        self.taylor = int(d.get("material", 0)) == 1
        self.coupled = self.taylor and bool(d.get("gnd_coupling", 0))
        self.relax = self.coupled and int(d.get("gnd_relax", 1)) == 1
        self.relax_omega0 = 0.5
        self.plane = bool(d.get("plane_stress", 0))
        if self.plane and self.grid.n[2] != 1:
            raise ValueError("plane stress needs a grid one voxel thick (N3 = 1)")
        self.tau0 = tau[self.gid].astype(np.float64)
        self.phi = np.zeros(M) if phi0 is None else np.asarray(phi0, dtype=float).copy()
        self.rho_ssd = np.full(M, d["rho0"])
        if self.taylor:
            self.g = self.tau0 + d["mu"] * d["burgers"] * np.sqrt(self.rho_ssd)
        else:
            self.g = self.tau0.copy()
        # voxels pre-set to full damage are the paper's geometric crack: a linear
        # elastic region (no slip) whose stiffness g(1) C = k C
        self.g[self.phi >= 1.0] = np.inf
        # optionally those voxels hold phi = 1 as a Dirichlet condition of the phase field
        self.preset = ~np.isfinite(self.g)
        self.pf_dirichlet = bool(d.get("pf_dirichlet", 0)) and bool(self.preset.any())
        self.rho_gnd = np.zeros(M)
        self.Wp = np.zeros(M)
        self.Gs = np.zeros(M)
        self.H = np.zeros(M)
        self.Wcrit = np.zeros(M)
        self.trig = np.zeros(M, dtype=bool)
        self.sig = np.zeros((M, 6))         # effective stress (Mandel), last converged
        self.sig_ws = None                  # warm start of the return map
        self.macro_sig = np.zeros(6)        # macro stress mean(g sigma) at t
        self.history = []

    # --- per-voxel constitutive update --------------------------------------------
    def constit(self, epsM, dt):
        t = self.tab
        gid = self.gid
        out = return_map(epsM, to_mandel2(self.epsp), self.g, dt, t.C[gid], t.S[gid],
                         t.P[gid], sig0=self.sig_ws, law=self.law)
        self.sig_ws = out[0]
        return out

    def degradation(self, phi):
        return (1.0 - phi) ** 2 + self.d["k_res"]

    # --- Algorithm 1 -------------------------------------------------------------
    def step(self, deps6, dt, dsig6=None, stress_mask=0):
        """One increment.  Components c (order xx, yy, zz, yz, xz, xy) with bit c set in
        stress_mask follow the macro stress increment dsig6[c] (mixed control); the
        others follow the macro strain increment deps6[c]."""
        d = self.d
        grid = self.grid
        t = self.tab
        gid = self.gid
        stats = {}
        free = [c for c in range(6) if (stress_mask >> c) & 1]
        de6 = np.array(deps6, dtype=float)
        if self.plane and (any(c in (2, 3, 4) for c in free) or np.any(de6[2:5] != 0.0)):
            raise ValueError("in plane stress the out-of-plane components are not controlled")
        de6[free] = 0.0
        dE = from_tensor6(de6)[0]
        target = self.macro_sig.copy()
        if free:
            target[free] += np.asarray(dsig6, dtype=float)[free]
        tgtM = to_mandel2(from_tensor6(target))[0]
        eps_t = self.eps.copy()
        phi_t = self.phi.copy()
        eps_prev = eps_t + dE[None]
        phi_prev = phi_t.copy()
        constit = lambda e: self.constit(e, dt)
        g_n = self.g.copy()
        slipping = np.isfinite(g_n)
        rho_gnd_new = self.rho_gnd
        omega, res_prev = self.relax_omega0, None
        mech = solve_mechanics_plane if self.plane else solve_mechanics
        for it in range(d["max_stag"]):
            eps_i, sig, dgam = mech(grid, eps_prev, eps_t, self.degradation(phi_prev), constit,
                                    d["tol_newton"], d["tol_lin"], d["max_newton"],
                                    d["max_krylov"], stats, free=free, sig_target=tgtM)
            epsp_tr = self.epsp + from_mandel2(np.einsum("ma,mai->mi", dgam, t.P[gid]))
            tau = np.einsum("mai,mi->ma", t.P[gid], sig)
            wp_tr = self.Wp + (tau * dgam).sum(1)
            we = we_plus(eps_i - epsp_tr, t.C4[gid])
            S = np.where(self.trig, d["ell"] / d["Gc"] * np.maximum(0.0, we + wp_tr - self.Wcrit),
                         0.0)
            if self.pf_dirichlet:
                phi_sol = solve_phase_field_dirichlet(grid, S, d["ell"], self.preset,
                                                      rtol=d["tol_lin"], max_iter=d["max_krylov"],
                                                      stats=stats)
            else:
                phi_sol = solve_phase_field(grid, S, d["ell"], x0=phi_prev, rtol=d["tol_lin"],
                                            max_iter=d["max_krylov"], stats=stats)
            phi_i = np.minimum(1.0, np.maximum(phi_t, phi_sol))
            r_e = _ratio(np.abs(tensor6(eps_i - eps_prev)).max(),
                         np.abs(tensor6(eps_i - eps_t)).max())
            r_p = _ratio(np.abs(phi_i - phi_prev).max(), np.abs(phi_i - phi_t).max())
            r_g = 0.0
            if self.coupled:
                # end-of-increment densities from this pass's slip, and the strength
                dbeta_i = np.einsum("ma,maij->mij", dgam, t.SN[gid])
                rho_ssd_new = self.rho_ssd + d["lambda_ssd"] * np.sqrt(
                    2.0 / 3.0 * np.einsum("mij,mij->m", dbeta_i, dbeta_i))
                lam_i = nye_tensor(grid, self.beta + dbeta_i, d["ell_fp"])
                rho_gnd_new = gnd_density(lam_i, t.R[gid], d["burgers"])
                g_new = np.where(slipping, self.tau0 + d["mu"] * d["burgers"] *
                                 np.sqrt(rho_ssd_new + rho_gnd_new), np.inf)
                r_g = _ratio(np.abs(g_new - self.g)[slipping].max(initial=0.0),
                             np.abs(g_new - g_n)[slipping].max(initial=0.0))
                if self.relax:
                    # Aitken's delta-squared relaxation of the fixed point g = T(g)
                    # (Irons and Tuck): residual r_i = T(g_i) - g_i over the slipping
                    # voxels, omega_i = -omega_(i-1) r_(i-1).(r_i - r_(i-1)) / |r_i - r_(i-1)|^2
                    res = np.where(slipping, g_new - self.g, 0.0)
                    if it > 0:
                        dr = res - res_prev
                        den = float((dr * dr).sum())
                        if den > 0.0:
                            omega = -omega * float((res_prev * dr).sum()) / den
                    res_prev = res
                    self.g = np.where(slipping, self.g + omega * res, np.inf)
                else:
                    self.g = g_new
            eps_prev, phi_prev = eps_i, phi_i
            stats["stag"] = it + 1
            if r_e <= d["tol_stag"] and r_p <= d["tol_stag"] and r_g <= d["tol_stag"]:
                break
        else:
            raise RuntimeError("alternating minimisation did not converge")
        # --- commit (all in float64) ---
        self.eps = eps_prev
        self.phi = phi_prev
        self.sig = sig
        dbeta = np.einsum("ma,maij->mij", dgam, t.SN[gid])
        self.epsp = epsp_tr
        self.beta = self.beta + dbeta
        if not self.taylor:
            self.g = self.g + d["h_lin"] * np.abs(dgam).sum(1)
        self.rho_ssd = self.rho_ssd + d["lambda_ssd"] * np.sqrt(
            2.0 / 3.0 * np.einsum("mij,mij->m", dbeta, dbeta))
        if self.coupled:
            self.rho_gnd = rho_gnd_new          # G_s with the end-of-increment GND density
        dw = (tau * dgam).sum(1)
        self.Wp = self.Wp + dw
        self.Gs = self.Gs + d["xi_store"] * dw / np.sqrt(self.rho_ssd + self.rho_gnd)
        self.H = np.maximum(self.H, we)
        newly = (~self.trig) & (self.Gs >= d["G_crit"])
        self.Wcrit = np.where(newly, self.H + self.Wp, self.Wcrit)
        self.trig = self.trig | newly
        lam = nye_tensor(grid, self.beta, d["ell_fp"])
        self.rho_gnd = gnd_density(lam, t.R[gid], d["burgers"])
        if self.taylor:
            self.g = np.where(np.isfinite(self.g), self.tau0 + d["mu"] * d["burgers"] *
                              np.sqrt(self.rho_ssd + self.rho_gnd), np.inf)
        gphi = self.degradation(self.phi)
        stats["macro_stress"] = tensor6((gphi[:, None, None] * from_mandel2(sig)).mean(0,
                                        keepdims=True))[0]
        self.macro_sig = stats["macro_stress"].copy()
        stats["macro_strain"] = tensor6(self.eps.mean(0, keepdims=True))[0]
        stats["max_phi"] = float(self.phi.max())
        stats["n_trig"] = int(self.trig.sum())
        self.history.append(stats)
        return stats

    # --- fields in the exchange layout ----------------------------------------------
    def fields(self):
        gphi = self.degradation(self.phi)
        sig_t = from_mandel2(self.sig)
        return dict(strain=tensor6(self.eps), stress=tensor6(gphi[:, None, None] * sig_t),
                    stress_eff=tensor6(sig_t), damage=self.phi.copy(), gs=self.Gs.copy(),
                    rho_ssd=self.rho_ssd.copy(), rho_gnd=self.rho_gnd.copy(), wp=self.Wp.copy(),
                    h=self.H.copy(), wcrit=self.Wcrit.copy(), trig=self.trig.astype(float),
                    eps_p=tensor6(self.epsp), g=self.g.copy())
