"""Finite-strain kinematics of the fatigue increment (oracle, test infrastructure).

Sec. 2.1 states the crystal plasticity in finite strain: F = Fe Fp with the plastic
velocity gradient Lp = dFp/dt Fp^-1 = sum_a gdot_a s_a (x) n_a; Sec. 3.1 (eqs. str1,
momentum, fdef, newton, precf, avstiff) balances the degraded first Piola-Kirchhoff
stress in the reference configuration with the deformation gradient F = F_bar + grad u,
grad u = F^-1{ u^ (x) i xi } (the i as in eq. newton), a 9 x 9 consistent tangent
K = dP/dF and the acoustic-tensor preconditioner [xi . Kbar . xi]^-1; eq. decMiehe
splits the Eulerian logarithmic elastic strain 1/2 ln(Fe Fe^T).

Readings (the paper names the kinematics, not their time integration):

* Elasticity: the second Piola-Kirchhoff stress of the intermediate (lattice)
  configuration is linear in the elastic Green-Lagrange strain, S = C : Ee,
  Ee = 1/2 (Fe^T Fe - I), with the cubic stiffness of the lattice (rotated by the grain
  orientation; the lattice keeps its reference orientation in that configuration).
* Backward Euler on the plastic deformation with the strength frozen over the step
  (as in the small-strain form), written as in Kalidindi, Bronkhorst and Anand (1992):
      A = Fe*^T Fe*, Fe* = F Fp_n^-1 (the trial elastic right Cauchy-Green tensor),
      Ee = 1/2 (A - I) - sum_a dgamma_a Q_a,   Q_a = sym(A s_a (x) n_a),
      tau_a = S : Q_a (the resolved shear of the Mandel stress of the trial state),
      dgamma_a = flow rule(tau_a, g),
  so that the stress S is the root of
      C^-1 : (S - S*) + sum_a dgamma_a(S : Q_a) Q_a = 0,   S* = C : 1/2 (A - I),
  the gradient of the strictly convex potential of the small-strain return map with the
  Schmid tensors P_a replaced by Q_a: the same unique root and the same Newton method.
  Then Fp_{n+1} = (I + sum_a dgamma_a s_a (x) n_a) Fp_n (the first-order exponential)
  and P = F Fp_{n+1}^-1 S Fp_{n+1}^-T.
* Plastic work per increment sum_a tau_a dgamma_a (tau from the converged S); the SSD
  rate lambda sqrt(2/3 dLp : dLp) with dLp = sum_a dgamma_a s_a (x) n_a; the Nye tensor
  is the regularised curl of Fp (the curl of the identity vanishes).
* eq. decMiehe: with Fe = F Fp_{n+1}^-1 and Fe = Ve Re, the Eulerian log strain ln Ve has
  the eigenvalues 1/2 ln(l_i) of Ce = Fe^T Fe and the eigenvectors Re N_i, where N_i are
  those of Ce; the lattice stiffness acts in the intermediate configuration, so
  W_e+ = 1/2 E+ : C : E+ with E+ = sum_i <1/2 ln l_i>+ N_i (x) N_i (the 1/2 of a strain
  energy density, as in the small-strain form).
* Newton for the momentum balance takes full steps, halving a step while the
  preconditioned residual grows (there is no incremental energy of this integration);
  it stops when max|grad du| <= tol max|F_i - F_t| (Sec. 3.1's criterion).  The
  operator is not symmetric, so the Krylov solver is the paper's GMRES.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, gmres

from .constitutive import GrainTables, return_map, flow_law
from .crystal import to_mandel2, from_mandel2, rotate4
from .spectral import Grid
from .phasefield import solve_phase_field, solve_phase_field_dirichlet
from .history import nye_tensor, gnd_density

EYE = np.eye(3)


def _sym(T):
    return 0.5 * (T + np.swapaxes(T, -1, -2))


def grad_hat(grid, uh):
    """Displacement gradient of eq. fdef: (u^ (x) i xi~)_ij = i xi~_j u^_i, (N..,3) -> (N..,3,3)."""
    return 1j * uh[..., :, None] * grid.xit[..., None, :]


def fs_return_map(F, Fp, g, dt, tab, gid, law, S0=None):
    """Finite-strain return map (readings above) at deformation gradients F (M,3,3).

    Fp: (M,3,3) plastic deformation at t_n; g: (M,) strength; tab: GrainTables; gid:
    (M,) grain ids; S0: optional warm start (M,6) Mandel.  Returns a dict with the
    second Piola-Kirchhoff stress S (Mandel, M x 6), dgam (M,12), its derivative ddg,
    the directions QM (M,12,6), the 6 x 6 Mandel K_S = dS/dEe*, P (M,3,3), Fp_new and
    the intermediate products the tangent needs.
    """
    Fp_inv = np.linalg.inv(Fp)
    Fe_tr = F @ Fp_inv
    A = np.swapaxes(Fe_tr, -1, -2) @ Fe_tr
    SN = tab.SN[gid]                                              # s (x) n, (M,12,3,3)
    QM = to_mandel2(_sym(np.einsum("mij,majk->maik", A, SN)))      # (M,12,6)
    Ee_tr = to_mandel2(0.5 * (A - EYE))
    S, dgam, KS, _ = return_map(Ee_tr, np.zeros_like(Ee_tr), g, dt, tab.C[gid], tab.S[gid],
                                QM, sig0=S0, law=law)
    tau = np.einsum("mai,mi->ma", QM, S)
    dgam, ddg = law.increments(tau, g, dt)
    dLp = np.einsum("ma,maij->mij", dgam, SN)
    X = EYE + dLp
    Xinv = np.linalg.inv(X)
    Fp_new = X @ Fp
    Gi = Fp_inv @ Xinv                                            # Fp_new^-1
    S2 = from_mandel2(S)
    P = F @ Gi @ S2 @ np.swapaxes(Gi, -1, -2)
    return dict(S=S, S2=S2, dgam=dgam, ddg=ddg, tau=tau, QM=QM, KS=KS, P=P, Fp_new=Fp_new,
                Gi=Gi, Xinv=Xinv, Fe_tr=Fe_tr, Fp_inv=Fp_inv, SN=SN, dLp=dLp)


def fs_tangent(F, r):
    """Consistent tangent K_ijkl = dP_ij / dF_kl (M,3,3,3,3) of fs_return_map's result r,
    by differentiating every step of the update (the root condition implicitly)."""
    M = len(F)
    K = np.empty((M, 3, 3, 3, 3))
    Gi, S2, Xinv = r["Gi"], r["S2"], r["Xinv"]
    GiT = np.swapaxes(Gi, -1, -2)
    for k in range(3):
        for l in range(3):
            dF = np.zeros((M, 3, 3))
            dF[:, k, l] = 1.0
            dA = 2.0 * _sym(np.swapaxes(r["Fe_tr"], -1, -2) @ dF @ r["Fp_inv"])
            dQM = to_mandel2(_sym(np.einsum("mij,majk->maik", dA, r["SN"])))
            s_dq = np.einsum("mi,mai->ma", r["S"], dQM)
            rhs = (to_mandel2(0.5 * dA)
                   - np.einsum("ma,mai->mi", r["ddg"] * s_dq, r["QM"])
                   - np.einsum("ma,mai->mi", r["dgam"], dQM))
            dS = np.einsum("mij,mj->mi", r["KS"], rhs)
            ddgam = r["ddg"] * (np.einsum("mai,mi->ma", r["QM"], dS) + s_dq)
            ddLp = np.einsum("ma,maij->mij", ddgam, r["SN"])
            dGi = -Gi @ ddLp @ Xinv
            dS2 = from_mandel2(dS)
            dP = (dF @ Gi @ S2 @ GiT + F @ dGi @ S2 @ GiT + F @ Gi @ dS2 @ GiT
                  + F @ Gi @ S2 @ np.swapaxes(dGi, -1, -2))
            K[:, :, :, k, l] = dP
    return K


def we_plus_log(Fe, C4):
    """eq. decMiehe with the logarithmic elastic strain: 1/2 E+ : C : E+ with
    E+ = sum_i <1/2 ln l_i>+ N_i (x) N_i over the eigenpairs of Ce = Fe^T Fe."""
    Ce = np.swapaxes(Fe, -1, -2) @ Fe
    lam, N = np.linalg.eigh(Ce)
    e = np.maximum(0.5 * np.log(lam), 0.0)
    Ep = np.einsum("mia,ma,mja->mij", N, e, N)
    return 0.5 * np.einsum("mij,mijkl,mkl->m", Ep, C4, Ep)


def fs_operator(grid, gK):
    """Linearised finite-strain momentum operator on flat real displacement vectors,
    matvec(u) = -F^-1{ i xi~_j F{ gK_ijkl F^-1{ i xi~_l u^_k } } }, and its preconditioner
    prec(r) = F^-1{ [xi~ . Kbar . xi~]^-1 F{r} }, Kbar = mean(gK) (eqs. newton, precf,
    avstiff).  gK: (M,3,3,3,3).  Returns (matvec, prec, count)."""
    n = grid.n
    Ainv = grid.acoustic_inverse(gK.mean(0))
    gK_g = grid.to_grid(gK)
    count = [0]

    def matvec(x):
        count[0] += 1
        u = x.reshape(n + (3,))
        dF = grid.ifft(grad_hat(grid, grid.fft(u)))
        dP = np.einsum("...ijkl,...kl->...ij", gK_g, dF)
        return -grid.ifft(grid.div_hat(grid.fft(dP))).ravel()

    def prec(x):
        y = np.einsum("...ik,...k->...i", Ainv, grid.fft(x.reshape(n + (3,))))
        return grid.ifft(y).ravel()

    return matvec, prec, count


def solve_mechanics_fs(grid, F0, F_t, gphi, constit, tol_newton, tol_lin, max_newton,
                       max_krylov, restart=200, stats=None):
    """Equilibrated deformation gradients (M,3,3) starting from F0.

    constit(F) -> (result dict of fs_return_map, K (M,3,3,3,3)).  Returns (F, result)."""
    n = grid.n
    gphi = np.asarray(gphi, dtype=np.float64)
    F = np.array(F0, dtype=np.float64, copy=True)
    r, K = constit(F)

    def residual(r_):
        gP = grid.to_grid(gphi[:, None, None] * r_["P"])
        return grid.ifft(grid.div_hat(grid.fft(gP))).ravel()

    rhs = residual(r)
    for it in range(max_newton):
        gK = gphi[:, None, None, None, None] * K
        matvec, prec, count = fs_operator(grid, gK)
        N = rhs.size
        A = LinearOperator((N, N), matvec=matvec, dtype=np.float64)
        Pm = LinearOperator((N, N), matvec=prec, dtype=np.float64)
        merit0 = np.linalg.norm(prec(rhs))
        du, info = gmres(A, rhs, M=Pm, rtol=tol_lin, atol=0.0, restart=restart,
                         maxiter=max_krylov)
        if info != 0:
            raise RuntimeError(f"finite-strain GMRES did not converge (info={info})")
        dF = grid.to_flat(grid.ifft(grad_hat(grid, grid.fft(du.reshape(n + (3,))))))
        t = 1.0
        for _ls in range(30):
            trial = F + t * dF
            r_t, K_t = constit(trial)
            rhs_t = residual(r_t)
            if np.linalg.norm(prec(rhs_t)) <= merit0 or merit0 == 0.0:
                break
            t *= 0.5
        else:
            raise RuntimeError("finite-strain Newton: no step reduces the residual")
        F, r, K, rhs = trial, r_t, K_t, rhs_t
        if stats is not None:
            stats["matvecs"] = stats.get("matvecs", 0) + count[0]
            stats["newton"] = stats.get("newton", 0) + 1
            stats["ls_cuts"] = stats.get("ls_cuts", 0) + _ls
        num = t * np.abs(dF).max()
        den = np.abs(F - F_t).max()
        if num <= tol_newton * den or num == 0.0:
            return F, r
    raise RuntimeError("finite-strain Newton did not converge")


def _ratio(num, den):
    if num == 0.0:
        return 0.0
    return num / den if den > 0.0 else np.inf


class OracleFiniteRVE:
    """State and increments (Algorithm 1) of one periodic RVE in finite strain.  ``desc``
    is the flat dict of ``synth.Workload.desc``; arrays are flat with x fastest."""

    def __init__(self, desc, grain, quat, tau_c0=None, phi0=None):
        self.d = dict(desc)
        d = self.d
        self.grid = Grid(d["n"], d["h"], 0)
        M = self.grid.M
        self.gid = np.asarray(grain, dtype=np.int64)
        quat = np.atleast_2d(np.asarray(quat, dtype=np.float64))
        self.tab = GrainTables(quat, d["C11"], d["C12"], d["C44"])
        G = len(quat)
        tau = np.full(G, d["tau_c0"]) if tau_c0 is None else np.asarray(tau_c0, dtype=float)
        self.law = flow_law(d)
        self.taylor = int(d.get("material", 0)) == 1
        self.tau0 = tau[self.gid].astype(np.float64)
        self.F = np.tile(EYE, (M, 1, 1))
        self.Fp = np.tile(EYE, (M, 1, 1))
        self.phi = np.zeros(M) if phi0 is None else np.asarray(phi0, dtype=float).copy()
        self.rho_ssd = np.full(M, d["rho0"])
        if self.taylor:
            self.g = self.tau0 + d["mu"] * d["burgers"] * np.sqrt(self.rho_ssd)
        else:
            self.g = self.tau0.copy()
        self.g[self.phi >= 1.0] = np.inf
        self.preset = ~np.isfinite(self.g)
        self.pf_dirichlet = bool(d.get("pf_dirichlet", 0)) and bool(self.preset.any())
        self.rho_gnd = np.zeros(M)
        self.Wp = np.zeros(M)
        self.Gs = np.zeros(M)
        self.H = np.zeros(M)
        self.Wcrit = np.zeros(M)
        self.trig = np.zeros(M, dtype=bool)
        self.S = np.zeros((M, 6))
        self.P = np.zeros((M, 3, 3))
        self.S_ws = None
        self.history = []

    def constit(self, F, dt):
        r = fs_return_map(F, self.Fp, self.g, dt, self.tab, self.gid, self.law, S0=self.S_ws)
        self.S_ws = r["S"]
        return r, fs_tangent(F, r)

    def degradation(self, phi):
        return (1.0 - phi) ** 2 + self.d["k_res"]

    def step(self, dF9, dt):
        """One increment under the macroscopic deformation gradient increment dF9 (3x3
        row-major, 9 values)."""
        d = self.d
        grid = self.grid
        t = self.tab
        gid = self.gid
        stats = {}
        dFbar = np.asarray(dF9, dtype=float).reshape(3, 3)
        F_t = self.F.copy()
        phi_t = self.phi.copy()
        F_prev = F_t + dFbar[None]
        phi_prev = phi_t.copy()
        constit = lambda F: self.constit(F, dt)
        C4 = t.C4[gid]
        for it in range(d["max_stag"]):
            F_i, r = solve_mechanics_fs(grid, F_prev, F_t, self.degradation(phi_prev), constit,
                                        d["tol_newton"], d["tol_lin"], d["max_newton"],
                                        d["max_krylov"], stats=stats)
            wp_tr = self.Wp + (r["tau"] * r["dgam"]).sum(1)
            we = we_plus_log(F_i @ r["Gi"], C4)
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
            r_F = _ratio(np.abs(F_i - F_prev).max(), np.abs(F_i - F_t).max())
            r_p = _ratio(np.abs(phi_i - phi_prev).max(), np.abs(phi_i - phi_t).max())
            F_prev, phi_prev = F_i, phi_i
            stats["stag"] = it + 1
            if r_F <= d["tol_stag"] and r_p <= d["tol_stag"]:
                break
        else:
            raise RuntimeError("alternating minimisation did not converge")
        # --- commit (all in float64) ---
        self.F = F_prev
        self.phi = phi_prev
        self.S = r["S"]
        self.P = r["P"]
        dgam = r["dgam"]
        self.Fp = r["Fp_new"]
        if not self.taylor:
            self.g = self.g + d["h_lin"] * np.abs(dgam).sum(1)
        dLp = r["dLp"]
        self.rho_ssd = self.rho_ssd + d["lambda_ssd"] * np.sqrt(
            2.0 / 3.0 * np.einsum("mij,mij->m", dLp, dLp))
        dw = (r["tau"] * dgam).sum(1)
        self.Wp = self.Wp + dw
        self.Gs = self.Gs + d["xi_store"] * dw / np.sqrt(self.rho_ssd + self.rho_gnd)
        self.H = np.maximum(self.H, we)
        newly = (~self.trig) & (self.Gs >= d["G_crit"])
        self.Wcrit = np.where(newly, self.H + self.Wp, self.Wcrit)
        self.trig = self.trig | newly
        lam = nye_tensor(grid, self.Fp, d["ell_fp"])
        self.rho_gnd = gnd_density(lam, t.R[gid], d["burgers"])
        if self.taylor:
            self.g = np.where(np.isfinite(self.g), self.tau0 + d["mu"] * d["burgers"] *
                              np.sqrt(self.rho_ssd + self.rho_gnd), np.inf)
        gphi = self.degradation(self.phi)
        stats["macro_stress"] = (gphi[:, None, None] * self.P).mean(0).ravel()
        stats["macro_defgrad"] = self.F.mean(0).ravel()
        stats["max_phi"] = float(self.phi.max())
        stats["n_trig"] = int(self.trig.sum())
        self.history.append(stats)
        return stats

    def fields(self):
        gphi = self.degradation(self.phi)
        M = self.grid.M
        return dict(defgrad=self.F.reshape(M, 9).copy(),
                    pk1=(gphi[:, None, None] * self.P).reshape(M, 9),
                    fp=self.Fp.reshape(M, 9).copy(), damage=self.phi.copy(), gs=self.Gs.copy(),
                    rho_ssd=self.rho_ssd.copy(), rho_gnd=self.rho_gnd.copy(), wp=self.Wp.copy(),
                    h=self.H.copy(), wcrit=self.Wcrit.copy(), trig=self.trig.astype(float),
                    g=self.g.copy())
