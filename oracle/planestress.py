"""Pointwise plane stress on one-voxel-thick plates (oracle, test infrastructure).

Sec. 4.1-4.3 model thin plates, N1 x N2 x 1 voxels with a thickness of one voxel, and
take them to be in plane stress.  The paper does not say how the condition enters the
FFT solve; the reading here is the generalised plane stress of a thin anisotropic
plate:
* the three out-of-plane stress components vanish at every voxel,
      sigma_zz = sigma_yz = sigma_xz = 0,
  so the out-of-plane strain components (zz, yz, xz) are free local unknowns rather
  than components of a compatible field;
* the in-plane strain is compatible: eps_p = E_p + sym grad (u_x, u_y), with the
  fields constant through the thickness (xi_z = 0 on an N3 = 1 grid), and the in-plane
  stress is divergence free;
* macroscopic control (strain, or the mixed control of mechanics.py) acts on the
  in-plane components xx, yy, xy only.

This oracle solves the condition as its definition states it: every constitutive
evaluation at a given in-plane strain first drives the out-of-plane stress to zero by
a local Newton iteration on the out-of-plane strain (with the out-of-plane block of the
consistent tangent), and the stiffness of the constrained point is the Schur
complement of that block, K_pp - K_po K_oo^-1 K_op.  The in-plane momentum balance is
then a two-dimensional problem solved like the three-dimensional one (mechanics.py:
Newton + conjugate gradients preconditioned by the inverse in-plane acoustic tensor,
backtracking on the incremental energy, which at the locally solved points is the
minimum of the energy over the out-of-plane strain, so that its gradient is the
in-plane stress).

Mandel index sets: in-plane P = (xx, yy, xy) = (0, 1, 5), out-of-plane
O = (zz, yz, xz) = (2, 3, 4).
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, cg

from .crystal import to_mandel2, from_mandel2, from_mandel4

P_IDX = np.array([0, 1, 5])
O_IDX = np.array([2, 3, 4])


def local_plane_stress(constit, epsM, rtol=1e-13, max_iter=60):
    """Out-of-plane strain at which the out-of-plane stress vanishes, per voxel.

    constit(eps_mandel) -> (sig, dgam, K, w).  The in-plane components of ``epsM``
    (M,6) are kept; the out-of-plane ones are the starting guess.  The point's
    incremental energy w is convex in the strain with gradient sigma, so the condition
    is the minimum of w over e_O: Newton steps d = -K_OO^-1 sigma_O, each voxel's step
    halved until w decreases by at least 1e-4 of the step's first-order change, until
    max|sigma_O| <= rtol max|sigma|.  Returns (epsM, sig, dgam, K, w) at the solution."""
    e = np.array(epsM, dtype=np.float64, copy=True)
    sig, dgam, K, w = constit(e)
    for _ in range(max_iter):
        so = sig[:, O_IDX]
        if np.abs(so).max() <= rtol * max(np.abs(sig).max(), 1e-300):
            return e, sig, dgam, K, w
        Koo = K[:, O_IDX][:, :, O_IDX]
        d = -np.linalg.solve(Koo, so[..., None])[..., 0]
        slope = (so * d).sum(1)
        s = np.ones(len(e))
        for _ls in range(60):
            trial = e.copy()
            trial[:, O_IDX] += s[:, None] * d
            out = constit(trial)
            bad = out[3] - w > 1e-4 * s * slope + 1e-13 * np.abs(w)
            if not bad.any():
                break
            s = np.where(bad, 0.5 * s, s)
        else:
            raise RuntimeError("local plane-stress line search failed")
        e = trial
        sig, dgam, K, w = out
    raise RuntimeError("local plane-stress iteration did not converge")


def condensed_tangent(K):
    """Stiffness of the point constrained to zero out-of-plane stress (M,3,3), in-plane
    Mandel order (xx, yy, xy): K_PP - K_PO K_OO^-1 K_OP."""
    Kpp = K[:, P_IDX][:, :, P_IDX]
    Kpo = K[:, P_IDX][:, :, O_IDX]
    Kop = K[:, O_IDX][:, :, P_IDX]
    Koo = K[:, O_IDX][:, :, O_IDX]
    return Kpp - Kpo @ np.linalg.solve(Koo, Kop)


def _inplane_strain(grid, u):
    """In-plane Mandel strain (M,3) of the displacement u (N1,N2,1,2) real."""
    uh = grid.fft(np.concatenate([u, np.zeros(u.shape[:-1] + (1,))], axis=-1))
    de = grid.to_flat(grid.ifft(grid.sym_grad_hat(uh)))
    return to_mandel2(de)[:, P_IDX]


def _inplane_div(grid, sP):
    """x, y components of -div of the in-plane stress (M,3 Mandel), as a flat vector."""
    s6 = np.zeros((sP.shape[0], 6))
    s6[:, P_IDX] = sP
    sh = grid.fft(grid.to_grid(from_mandel2(s6)))
    return -grid.ifft(grid.div_hat(sh))[..., :2].ravel()


def plane_operator(grid, gKc):
    """Linearised in-plane momentum operator -div(gKc : sym grad du) on flat (u_x, u_y)
    vectors and its preconditioner [xi~ . Kbar . xi~]^-1 restricted to x, y, with Kbar
    the mean condensed tangent (the plate's eq. precf)."""
    n = grid.n
    K6 = np.zeros((6, 6))
    K6[np.ix_(P_IDX, P_IDX)] = gKc.mean(0)
    K4 = from_mandel4(K6)
    A = np.einsum("...j,ijkl,...l->...ik", grid.xit, K4, grid.xit)[..., :2, :2]
    Ainv = np.zeros_like(A)
    nz = grid.nonzero
    Ainv[nz] = np.linalg.inv(A[nz])
    count = [0]

    def matvec(x):
        count[0] += 1
        dP = _inplane_strain(grid, x.reshape(n + (2,)))
        return _inplane_div(grid, np.einsum("mij,mj->mi", gKc, dP))

    def prec(x):
        y = np.einsum("...ik,...k->...i", Ainv, grid.fft(x.reshape(n + (2,))))
        return grid.ifft(y).ravel()

    return matvec, prec, count


def solve_mechanics_plane(grid, eps0, eps_t, gphi, constit, tol_newton, tol_lin, max_newton,
                          max_krylov, stats=None, free=(), sig_target=None):
    """Equilibrated strain (M,3,3) of a plate in pointwise plane stress from ``eps0``
    (whose out-of-plane components start the local iterations).

    free: Mandel indices among (0, 1, 5) under macro stress control, sig_target (6,)
    Mandel.  The stop test is the paper's: max|eps_(i+1) - eps_i| <= tol_newton
    max|eps_(i+1) - eps_t| over all components.  Returns (eps, sig_mandel, dgam)."""
    assert grid.n[2] == 1
    free = [int(c) for c in sorted(free)]
    assert all(c in (0, 1, 5) for c in free)
    fp = np.array([list(P_IDX).index(c) for c in free], dtype=np.int64)   # in-plane slots
    nf = len(fp)
    gphi = np.asarray(gphi, dtype=np.float64)
    M = len(gphi)
    tgt = np.zeros(6) if sig_target is None else np.asarray(sig_target, dtype=np.float64)
    tgtP = tgt[P_IDX]
    ext = lambda eM: -tgtP[fp] @ eM[:, P_IDX].mean(0)[fp] if nf else 0.0
    eM, sigM, dgam, KM, w = local_plane_stress(constit, to_mandel2(eps0))
    Pi = np.mean(gphi * w) + ext(eM)
    n = grid.n
    for it in range(max_newton):
        gKc = gphi[:, None, None] * condensed_tangent(KM)
        matvec, prec, count = plane_operator(grid, gKc)
        gsP = gphi[:, None] * sigM[:, P_IDX]
        rhs = -_inplane_div(grid, gsP)
        Nu = rhs.size
        if nf:
            Kff_inv = np.linalg.inv(gKc.sum(0)[np.ix_(fp, fp)])
            rhs = np.concatenate([rhs, -(gsP.sum(0)[fp] - M * tgtP[fp])])

            def mv(x, matvec=matvec, gKc=gKc):
                u, dE = x[:Nu], x[Nu:]
                E3 = np.zeros(3)
                E3[fp] = dE
                sE = np.einsum("mij,j->mi", gKc, E3)
                fl = matvec(u) + _inplane_div(grid, sE)
                tot = _inplane_strain(grid, u.reshape(n + (2,))) + E3[None]
                mac = np.einsum("mij,mj->i", gKc, tot)[fp]
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
        deP = _inplane_strain(grid, sol[:Nu].reshape(n + (2,)))
        if nf:
            deP[:, fp] += sol[Nu:][None]
        slope = np.mean(gphi * np.einsum("mi,mi->m", sigM[:, P_IDX], deP))
        if nf:
            slope -= tgtP[fp] @ deP.mean(0)[fp]
        t = 1.0
        for _ls in range(40):
            trial = eM.copy()
            trial[:, P_IDX] += t * deP
            e_t, s_t, dg_t, K_t, w_t = local_plane_stress(constit, trial)
            Pi_t = np.mean(gphi * w_t) + ext(e_t)
            if Pi_t - Pi <= 1e-4 * t * slope + 1e-13 * abs(Pi):
                break
            t *= 0.5
        else:
            raise RuntimeError("Newton line search failed")
        step = np.abs(from_mandel2(e_t) - from_mandel2(eM)).max()
        eM, sigM, dgam, KM, Pi = e_t, s_t, dg_t, K_t, Pi_t
        if stats is not None:
            stats["matvecs"] = stats.get("matvecs", 0) + count[0]
            stats["newton"] = stats.get("newton", 0) + 1
            stats["ls_cuts"] = stats.get("ls_cuts", 0) + _ls
        den = np.abs(from_mandel2(eM) - eps_t).max()
        if step <= tol_newton * den or step == 0.0:
            return from_mandel2(eM), sigM, dgam
    raise RuntimeError("Newton did not converge")
