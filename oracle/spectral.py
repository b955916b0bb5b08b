"""Fourier-space operators on the periodic voxel grid (oracle, test infrastructure).

Sec. 3.1: fields live at voxel centres of an N1 x N2 x N3 grid with edge h;
the frequency vectors are xi_a = 2 pi m_a / L_a over the DFT index set (the
paper's centred enumeration is the same set).  Spatial derivatives become
multiplications by i xi (eqs. momentum, phase, fdef, newton and the Nye
curl).

Reading used for the odd-order derivatives: on an even axis the Nyquist
index has no real-valued derivative, so gradient, divergence, curl and the
acoustic tensor use xi~, which is xi with that index set to zero.  The
Laplacian (phase field and regulariser) uses |xi|^2 with the Nyquist index
kept.

Optional discrete derivative (the remedy for Gibbs oscillations that Sec. 3.1 names:
discrete derivative definitions): the rotated scheme replaces i xi~_a by the symbol of a
forward difference along a averaged over the four parallel voxel edges,
    k_a = D(theta_a) prod_{b != a} A(theta_b),
    D(theta) = (e^{i theta} - 1) / h,   A(theta) = (1 + e^{i theta}) / 2,
theta_b = 2 pi m_b / N_b (A = 0 exactly at the Nyquist index).  Gradient sym(k (x) u^),
its adjoint conj(k) . sigma^ and the acoustic tensor conj(k) . K . k follow; the
Laplacian and the Nye curl stay spectral.

The oracle uses full complex FFTs of real fields (scipy.fft.fftn / ifftn);
per-voxel arrays are flat with x fastest, converted to (N1, N2, N3, ...)
grids for the transforms.
"""
import os
import numpy as np
import scipy.fft as sfft

WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


class Grid:
    def __init__(self, n, h, scheme=0):
        self.n = tuple(int(v) for v in n)
        self.h = float(h)
        self.scheme = int(scheme)          # 0: spectral (i xi~), 1: rotated differences
        self.M = int(np.prod(self.n))
        xi, xit = [], []
        for N in self.n:
            m = np.fft.fftfreq(N, 1.0 / N)               # integer frequency numbers
            L = N * self.h
            k = 2.0 * np.pi * m / L
            kt = k.copy()
            if N % 2 == 0:
                kt[N // 2] = 0.0
            xi.append(k)
            xit.append(kt)
        g = np.meshgrid(*xi, indexing="ij")
        gt = np.meshgrid(*xit, indexing="ij")
        self.xi = np.stack(g, axis=-1)                   # (N1,N2,N3,3), Laplacian symbol
        self.xit = np.stack(gt, axis=-1)                 # (N1,N2,N3,3), odd derivatives
        self.xi2 = (self.xi ** 2).sum(-1)
        self.nonzero = (self.xit ** 2).sum(-1) > 0
        if self.scheme == 1:
            D, A = [], []
            for N in self.n:
                m = np.arange(N)
                e = np.exp(2j * np.pi * m / N)
                e[0] = 1.0
                if N % 2 == 0:
                    e[N // 2] = -1.0
                D.append((e - 1.0) / self.h)
                A.append(0.5 * (1.0 + e))
            Dg = np.meshgrid(*D, indexing="ij")
            Ag = np.meshgrid(*A, indexing="ij")
            self.k = np.stack([Dg[0] * Ag[1] * Ag[2], Ag[0] * Dg[1] * Ag[2],
                               Ag[0] * Ag[1] * Dg[2]], axis=-1)
            self.nonzero = (np.abs(self.k) ** 2).sum(-1) > 0

    # --- layout -----------------------------------------------------------------
    def to_grid(self, f):
        """(M, ...) flat x-fastest -> (N1, N2, N3, ...)."""
        n1, n2, n3 = self.n
        f = np.asarray(f)
        rest = f.shape[1:]
        return np.moveaxis(f.reshape((n3, n2, n1) + rest), (0, 1, 2), (2, 1, 0))

    def to_flat(self, a):
        """(N1, N2, N3, ...) -> (M, ...) flat x-fastest."""
        rest = a.shape[3:]
        return np.moveaxis(a, (0, 1, 2), (2, 1, 0)).reshape((self.M,) + rest)

    # --- transforms -------------------------------------------------------------
    def fft(self, a):
        return sfft.fftn(a, axes=(0, 1, 2), workers=WORKERS)

    def ifft(self, a):
        return sfft.ifftn(a, axes=(0, 1, 2), workers=WORKERS).real

    # --- operators (grid arrays) --------------------------------------------------
    def sym_grad_hat(self, uh):
        """sym(i xi~ (x) u^) : (N..,3) complex -> (N..,3,3) complex (rotated scheme:
        sym(k (x) u^))."""
        if self.scheme == 1:
            g = self.k[..., :, None] * uh[..., None, :]
            return 0.5 * (g + np.swapaxes(g, -1, -2))
        g = 1j * self.xit[..., :, None] * uh[..., None, :]     # i xi_i u_j
        return 0.5 * (g + np.swapaxes(g, -1, -2))

    def div_hat(self, sh):
        """i xi~_j sigma^_ij : (N..,3,3) -> (N..,3) (rotated scheme: -conj(k_j) sigma^_ij,
        minus the adjoint of the gradient, as i xi~ = -conj(i xi~))."""
        if self.scheme == 1:
            return -np.einsum("...ij,...j->...i", sh, np.conj(self.k))
        return np.einsum("...ij,...j->...i", sh, 1j * self.xit)

    def acoustic_inverse(self, K4):
        """[xi~ . K . xi~]^-1 per frequency (zero where xi~ = 0), eq. precf (rotated
        scheme: [conj(k) . K . k]^-1, zero where k = 0)."""
        if self.scheme == 1:
            A = np.einsum("...j,ijkl,...l->...ik", np.conj(self.k), K4, self.k)
            Ainv = np.zeros_like(A)
            nz = self.nonzero
            Ainv[nz] = np.linalg.inv(A[nz])
            return Ainv
        A = np.einsum("...j,ijkl,...l->...ik", self.xit, K4, self.xit)
        Ainv = np.zeros_like(A)
        nz = self.nonzero
        Ainv[nz] = np.linalg.inv(A[nz])
        return Ainv

    def curl_hat(self, bh):
        """Row-wise curl: Lambda^_ij = eps_jkl i xi~_k beta^_il (Fourier form of nye1)."""
        e = np.zeros((3, 3, 3))
        e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1.0
        e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1.0
        return np.einsum("jkl,...k,...il->...ij", e, 1j * self.xit, bh)
