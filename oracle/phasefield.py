"""Phase-field damage: spectral split, driving state and the AT2 balance (oracle).

eq. decMiehe: the tensile part of the elastic strain, eps+ = sum <e_i>_+ n_i (x) n_i,
read in small strain as the eigen-decomposition of eps_e = eps - eps_p, and the
tensile energy read as the strain energy density 1/2 eps+ : C : eps+.
eq. zeta: S = (l W_crit / Gc) <(W_e+ + W_p) / W_crit - 1> = (l / Gc) <W - W_crit>
once the stored-energy threshold has been reached (zero before).
eqs. strpf / phase: (phi - l^2 lap phi) - 2 (1 - phi) S = 0, i.e.
    (1 + 2S) phi - l^2 lap phi = 2S,
solved here by conjugate gradients (the operator is symmetric positive definite)
with the preconditioner of eq. precph read as F^-1{ (1 + l^2 |xi|^2)^-1 F{.} }.
Optionally the pre-set crack voxels hold phi = 1 as a Dirichlet condition of the balance
(instead of entering it as free unknowns that the clamp to [phi_t, 1] resets).
"""
import numpy as np
from scipy.sparse.linalg import LinearOperator, cg


def split_positive(E):
    """Positive spectral part of symmetric tensors E (M,3,3)."""
    w, v = np.linalg.eigh(E)
    wp = np.maximum(w, 0.0)
    return np.einsum("mia,ma,mja->mij", v, wp, v)


def we_plus(E, C4):
    """1/2 eps+ : C : eps+ with eps+ the positive part of E; C4 (M,3,3,3,3)."""
    Ep = split_positive(E)
    return 0.5 * np.einsum("mij,mijkl,mkl->m", Ep, C4, Ep)


def solve_phase_field_dirichlet(grid, S, ell, fixed, rtol=1e-12, max_iter=2000, stats=None):
    """The same balance with phi = 1 held on the voxels of the boolean mask ``fixed`` (a
    pre-set crack as a Dirichlet condition): phi = u + 1_fixed with u = 0 on ``fixed`` and,
    on the free voxels F, P A P u = P (2S - A 1_fixed), A = (1 + 2S) - l^2 lap, P the
    restriction to F; conjugate gradients with the restricted preconditioner
    P (1 + l^2 |xi|^2)^-1 P (symmetric positive definite on F)."""
    S = np.asarray(S, dtype=np.float64)
    n = grid.n
    free = grid.to_grid(~np.asarray(fixed, dtype=bool)).astype(np.float64).ravel()
    phiD = 1.0 - free
    S_g = grid.to_grid(S).ravel()
    sym = 1.0 + ell ** 2 * grid.xi2
    count = [0]

    def lap_op(x):                       # -l^2 lap x
        return grid.ifft(ell ** 2 * grid.xi2 * grid.fft(x.reshape(n))).ravel()

    def matvec(x):
        count[0] += 1
        u = free * x
        return free * ((1.0 + 2.0 * S_g) * u + lap_op(u))

    def prec(x):
        return free * grid.ifft(grid.fft((free * x).reshape(n)) / sym).ravel()

    rhs = free * (2.0 * S_g - ((1.0 + 2.0 * S_g) * phiD + lap_op(phiD)))
    N = S.size
    A = LinearOperator((N, N), matvec=matvec, dtype=np.float64)
    P = LinearOperator((N, N), matvec=prec, dtype=np.float64)
    u, info = cg(A, rhs, rtol=rtol, atol=0.0, maxiter=max_iter, M=P)
    if info != 0:
        raise RuntimeError(f"phase-field CG did not converge (info={info})")
    if stats is not None:
        stats["pf_iters"] = stats.get("pf_iters", 0) + count[0]
    return grid.to_flat((free * u + phiD).reshape(n))


def solve_phase_field(grid, S, ell, x0=None, rtol=1e-12, max_iter=2000, stats=None):
    """Solve (1 + 2S) phi - l^2 lap phi = 2S on the periodic grid; S (M,) flat."""
    S = np.asarray(S, dtype=np.float64)
    b = 2.0 * S
    if not np.any(b):
        return np.zeros_like(S)
    n = grid.n
    S_g = grid.to_grid(S)
    sym = 1.0 + ell ** 2 * grid.xi2
    count = [0]

    def matvec(x):
        count[0] += 1
        f = x.reshape(n)
        lap_term = grid.ifft(ell ** 2 * grid.xi2 * grid.fft(f))    # -l^2 lap f
        return ((1.0 + 2.0 * S_g) * f + lap_term).ravel()

    def prec(x):
        return grid.ifft(grid.fft(x.reshape(n)) / sym).ravel()

    A = LinearOperator((S.size, S.size), matvec=matvec, dtype=np.float64)
    P = LinearOperator((S.size, S.size), matvec=prec, dtype=np.float64)
    start = None if x0 is None else grid.to_grid(x0).ravel()
    phi, info = cg(A, grid.to_grid(b).ravel(), x0=start, rtol=rtol, atol=0.0,
                   maxiter=max_iter, M=P)
    if info != 0:
        raise RuntimeError(f"phase-field CG did not converge (info={info})")
    if stats is not None:
        stats["pf_iters"] = stats.get("pf_iters", 0) + count[0]
    return grid.to_flat(phi.reshape(n))
