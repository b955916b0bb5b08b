"""Nye tensor and GND density (oracle, test infrastructure).

Sec. 3.1: the plastic distortion is regularised by solving
    beta~ - l_Fp^2 lap beta~ = beta      (read with l_Fp squared, so the
                                          equation is dimensionally consistent)
in Fourier space, and the Nye tensor is its curl (eq. nye1 and its Fourier
form), Lambda_ij = eps_jkl d_k beta~_il.  In the crystal frame Lambda_c =
R^T Lambda R is split into 12 edge and 6 screw densities by the minimum-norm
(L2) solution rho = A^+ vec(Lambda_c) / b, and rho_GND = ||rho||_2 (eq. for
rho_GND).
"""
import numpy as np

from .crystal import gnd_matrix


def nye_tensor(grid, beta, ell_fp):
    """beta (M,3,3) flat -> regularised Nye tensor (M,3,3)."""
    bh = grid.fft(grid.to_grid(beta))
    bh = bh / (1.0 + ell_fp ** 2 * grid.xi2)[..., None, None]
    return grid.to_flat(grid.ifft(grid.curl_hat(bh)))


def gnd_density(lam, R, burgers):
    """Scalar GND density from the Nye tensor (M,3,3) and per-voxel rotations (M,3,3)."""
    lam_c = np.einsum("mai,mab,mbj->mij", R, lam, R)          # R^T Lambda R
    Apinv = np.linalg.pinv(gnd_matrix())                     # 18 x 9
    rho = np.einsum("ki,mi->mk", Apinv, lam_c.reshape(len(lam_c), 9)) / burgers
    return np.linalg.norm(rho, axis=1)
