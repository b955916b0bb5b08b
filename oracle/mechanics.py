"""Momentum balance at fixed damage: Newton + Krylov in Fourier space (oracle).

Sec. 3.1, eqs. momentum, fdef, newton, precf, avstiff (small strain):
find the displacement fluctuation u such that, with
    eps = eps_bar + F^-1{ sym(i xi~ (x) u^) },
the degraded stress g(phi) sigma(eps) is divergence free on every frequency
with xi~ != 0.  Each Newton step solves the linearised balance
    - i xi~ . F{ g K : F^-1{ sym(i xi~ (x) du^) } } = i xi~ . F{ g sigma }
preconditioned by M = [xi~ . Kbar . xi~]^-1, Kbar = mean(g K) (eq. precf).

Readings:
* With the strength frozen over the step the tangent K is symmetric positive
  definite, so the linearised operator is symmetric positive definite and the
  Krylov solver is preconditioned conjugate gradients (the paper names GMRES;
  both converge to the same Newton correction).
* The unknown here is the real displacement correction field (the paper's
  real-FFT reduction is a change of basis of the same real vector space).
* Newton is globalised by backtracking on the convex incremental energy
  Pi(u) = mean(g w(eps(u))), whose gradient is the residual; the converged
  state is the same equilibrium, and full steps are taken near it.
* Newton stops when max|sym grad du| <= tol * max|eps_i - eps_t| (the paper's
  criterion, with the applied step).

Mixed control (the DBFFT mixed extension the paper relies on, Sec. 3.1): for the
macroscopic components in ``free`` (Mandel indices) the macro stress mean(g sigma) is
prescribed (``sig_target``, Mandel) and the macro strain E_F is an unknown.  The Newton
system gains those unknowns; with
    eps = E + eps~(u),
the linearised operator on (du, dE_F) is the Hessian of
    Pi(u, E_F) = sum_v g w(eps) - N sig_target . E_F,
    [ -div(gK : (eps~(du) + dE)) ;  sum_v (gK : (eps~(du) + dE))_F ],
symmetric positive definite in the Euclidean inner product (spectral gradient and
divergence are negative adjoints), preconditioned block-diagonally by the inverse
acoustic tensor and (N Kbar_FF)^-1.
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, cg

from .crystal import to_mandel2, from_mandel2, from_mandel4


def momentum_operator(grid, gK):
    """The linearised momentum operator and its preconditioner for a tangent field.

    gK: (M,6,6) Mandel degraded tangent g(phi) K.  Returns (matvec, prec, count):
    matvec(u) = -F^-1{ i xi~ . F{ gK : F^-1{ sym(i xi~ (x) F{u}) } } } on flat real
    displacement vectors, prec(r) = F^-1{ [xi~ . Kbar . xi~]^-1 F{r} } with Kbar =
    mean(gK), and count[0] the number of operator applications so far.
    """
    n = grid.n
    Ainv = grid.acoustic_inverse(from_mandel4(gK.mean(0)))
    gK_g = grid.to_grid(gK)
    count = [0]

    def matvec(x):
        count[0] += 1
        u = x.reshape(n + (3,))
        de = grid.ifft(grid.sym_grad_hat(grid.fft(u)))
        ds = from_mandel2(np.einsum("...ij,...j->...i", gK_g, to_mandel2(de)))
        return -grid.ifft(grid.div_hat(grid.fft(ds))).ravel()

    def prec(x):
        y = np.einsum("...ik,...k->...i", Ainv, grid.fft(x.reshape(n + (3,))))
        return grid.ifft(y).ravel()

    return matvec, prec, count


def solve_mechanics(grid, eps0, eps_t, gphi, constit, tol_newton, tol_lin, max_newton,
                    max_krylov, stats=None, free=(), sig_target=None):
    """Equilibrated strain (M,3,3) starting from ``eps0``.

    constit(eps_mandel) -> (sig_mandel, dgam, K_mandel, w) is the per-voxel update.
    gphi: (M,) degradation g(phi).  free: Mandel indices of the macro components under
    stress control, sig_target: (6,) Mandel macro stress they must reach.  Returns
    (eps, sig_mandel, dgam) at the solution.
    """
    n = grid.n
    free = np.asarray(sorted(free), dtype=np.int64)
    nf = len(free)
    gphi = np.asarray(gphi, dtype=np.float64)
    eps = np.array(eps0, dtype=np.float64, copy=True)
    sigM, dgam, KM, w = constit(to_mandel2(eps))
    M = len(gphi)
    tgt = np.zeros(6) if sig_target is None else np.asarray(sig_target, dtype=np.float64)
    # external work of the prescribed macro stress: - N sig_target . E_F, as a mean
    ext = lambda e: -tgt[free] @ to_mandel2(e).mean(0)[free] if nf else 0.0
    Pi = np.mean(gphi * w) + ext(eps)
    for it in range(max_newton):
        gKM = gphi[:, None, None] * KM
        matvec, prec, count = momentum_operator(grid, gKM)
        gsig = grid.to_grid(gphi[:, None, None] * from_mandel2(sigM))
        rhs = grid.ifft(grid.div_hat(grid.fft(gsig))).ravel()
        Nu = rhs.size
        if nf:
            sumK = gKM.sum(0)
            Kff_inv = np.linalg.inv(sumK[np.ix_(free, free)])
            gsigM = gphi[:, None] * sigM
            rhs = np.concatenate([rhs, -(gsigM.sum(0)[free] - M * tgt[free])])
            gK_g = grid.to_grid(gKM)

            def mv(x, matvec=matvec, gKM=gKM, gK_g=gK_g):
                u, dE = x[:Nu], x[Nu:]
                E6 = np.zeros(6)
                E6[free] = dE
                # fluctuation rows: -div(gK : (eps~(u) + dE)) = matvec(u) - div(gK : dE)
                sE = from_mandel2(np.einsum("...ij,j->...i", gK_g, E6))
                fl = matvec(u) - grid.ifft(grid.div_hat(grid.fft(sE))).ravel()
                de = grid.to_flat(grid.ifft(grid.sym_grad_hat(grid.fft(u.reshape(n + (3,))))))
                tot = to_mandel2(de) + E6[None]
                mac = np.einsum("mij,mj->i", gKM, tot)[free]
                return np.concatenate([fl, mac])

            def pc(x, prec=prec, Kff_inv=Kff_inv):
                return np.concatenate([prec(x[:Nu]), Kff_inv @ x[Nu:]])

            A = LinearOperator((Nu + nf, Nu + nf), matvec=mv, dtype=np.float64)
            P = LinearOperator((Nu + nf, Nu + nf), matvec=pc, dtype=np.float64)
        else:
            A = LinearOperator((Nu, Nu), matvec=matvec, dtype=np.float64)
            P = LinearOperator((Nu, Nu), matvec=prec, dtype=np.float64)
        sol, info = cg(A, rhs, rtol=tol_lin, atol=0.0, maxiter=max_krylov, M=P)
        if info != 0:
            raise RuntimeError(f"Krylov solve did not converge (info={info})")
        du = sol[:Nu]
        de = grid.to_flat(grid.ifft(grid.sym_grad_hat(grid.fft(du.reshape(n + (3,))))))
        if nf:
            E6 = np.zeros(6)
            E6[free] = sol[Nu:]
            de = de + from_mandel2(E6[None])
        # backtracking on the incremental energy along de
        slope = np.mean(gphi * np.einsum("mi,mi->m", sigM, to_mandel2(de))) + \
            (ext(de) if nf else 0.0)
        t = 1.0
        for _ls in range(40):
            trial = eps + t * de
            s_t, dg_t, K_t, w_t = constit(to_mandel2(trial))
            Pi_t = np.mean(gphi * w_t) + ext(trial)
            if Pi_t - Pi <= 1e-4 * t * slope + 1e-13 * abs(Pi):
                break
            t *= 0.5
        else:
            raise RuntimeError("Newton line search failed")
        eps = trial
        sigM, dgam, KM, Pi = s_t, dg_t, K_t, Pi_t
        if stats is not None:
            stats["matvecs"] = stats.get("matvecs", 0) + count[0]
            stats["newton"] = stats.get("newton", 0) + 1
            stats["ls_cuts"] = stats.get("ls_cuts", 0) + _ls
        num = t * np.abs(de).max()
        den = np.abs(eps - eps_t).max()
        if num <= tol_newton * den or num == 0.0:
            return eps, sigM, dgam
    raise RuntimeError("Newton did not converge")
