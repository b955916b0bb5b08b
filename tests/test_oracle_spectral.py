"""Pins of the oracle's Fourier machinery against brute force, closed forms and invariants
(Sec. 3.1: frequency vectors, Fourier derivatives, the preconditioner of eq. precf)."""
import numpy as np
import pytest

from oracle import Grid, cubic_stiffness
from oracle.crystal import to_mandel4


def brute_dft(a):
    """O(N^6) DFT: A(m) = sum_x a(x) exp(-2 pi i m.x / N)."""
    n1, n2, n3 = a.shape
    out = np.zeros(a.shape, dtype=complex)
    x = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    for m1 in range(n1):
        for m2 in range(n2):
            for m3 in range(n3):
                ph = m1 * x[..., 0] / n1 + m2 * x[..., 1] / n2 + m3 * x[..., 2] / n3
                out[m1, m2, m3] = (a * np.exp(-2j * np.pi * ph)).sum()
    return out


@pytest.mark.parametrize("n", [(4, 4, 4), (3, 3, 3), (6, 4, 3), (2, 6, 5)])
def test_fft_matches_bruteforce_dft(n):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(n)
    g = Grid(n, 1.0)
    ref = brute_dft(a)
    assert np.abs(g.fft(a) - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(g.ifft(ref) - a).max() <= 1e-14 * np.abs(a).max() * 10


def test_frequency_set_matches_centred_enumeration():
    # the paper enumerates xi = 2 pi (n - floor(N/2)) / L for n = 0..N-1
    for N in (4, 5, 6, 16):
        g = Grid((N, 2, 2), 0.5)
        L = N * 0.5
        paper = sorted(2 * np.pi * (np.arange(N) - N // 2) / L)
        ours = sorted(g.xi[:, 0, 0, 0])
        assert np.allclose(ours, paper, rtol=0, atol=1e-12)
        if N % 2 == 0:
            assert g.xit[N // 2, 0, 0, 0] == 0.0


def test_gradient_of_plane_wave_closed_form():
    # u_y = A sin(2 pi x / L): eps_xy = (A/2) (2 pi / L) cos(2 pi x / L), others zero
    n, h, A = (8, 4, 4), 0.3, 0.01
    g = Grid(n, h)
    L = n[0] * h
    x = (np.arange(n[0]) + 0.5) * h
    u = np.zeros(n + (3,))
    u[..., 1] = A * np.sin(2 * np.pi * x / L)[:, None, None]
    e = g.ifft(g.sym_grad_hat(g.fft(u)))
    exact = 0.5 * A * 2 * np.pi / L * np.cos(2 * np.pi * x / L)
    assert np.allclose(e[..., 0, 1], exact[:, None, None], atol=1e-15)
    assert np.allclose(e[..., 1, 0], exact[:, None, None], atol=1e-15)
    e2 = e.copy()
    e2[..., 0, 1] = e2[..., 1, 0] = 0
    assert np.abs(e2).max() < 1e-15


def test_divergence_is_minus_adjoint_of_gradient():
    # discrete integration by parts: <sym grad u, s> = -<u, div s> for real periodic fields
    rng = np.random.default_rng(2)
    n = (6, 4, 8)
    g = Grid(n, 1.3)
    u = rng.standard_normal(n + (3,))
    s = rng.standard_normal(n + (3, 3))
    s = 0.5 * (s + np.swapaxes(s, -1, -2))
    e = g.ifft(g.sym_grad_hat(g.fft(u)))
    d = g.ifft(g.div_hat(g.fft(s)))
    lhs = (e * s).sum()
    rhs = -(u * d).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # fields built from real inputs stay real
    assert np.abs(np.fft.ifftn(g.sym_grad_hat(g.fft(u)), axes=(0, 1, 2)).imag).max() < 1e-14


def _green_projector(g, K4):
    """Gamma(K): eps -> sym grad of the displacement that equilibrates K : eps."""
    Ainv = g.acoustic_inverse(K4)

    def P(e):
        s = np.einsum("ijkl,...kl->...ij", K4, e)
        uh = -np.einsum("...ik,...k->...i", Ainv, g.div_hat(g.fft(s)))
        return g.ifft(g.sym_grad_hat(uh))
    return P


def test_green_projection_idempotent_and_complement_equilibrated():
    rng = np.random.default_rng(3)
    n = (6, 6, 4)
    g = Grid(n, 1.0)
    K4 = cubic_stiffness(168.4e9, 121.4e9, 75.4e9)
    P = _green_projector(g, K4)
    x = rng.standard_normal(n + (3, 3))
    x = 0.5 * (x + np.swapaxes(x, -1, -2))
    x -= x.mean(axis=(0, 1, 2))
    px = P(x)
    assert np.abs(P(px) - px).max() <= 1e-13 * np.abs(px).max()
    # a compatible field is reproduced
    u = rng.standard_normal(n + (3,))
    e = g.ifft(g.sym_grad_hat(g.fft(u)))
    assert np.abs(P(e) - e).max() <= 1e-13 * np.abs(e).max()
    # the complement is K-equilibrated
    r = np.einsum("ijkl,...kl->...ij", K4, x - px)
    div = g.div_hat(g.fft(r))
    assert np.abs(div).max() <= 1e-12 * np.abs(g.fft(r)).max() * np.abs(g.xit).max()


def test_acoustic_tensor_of_isotropic_medium_closed_form():
    # isotropic: xi.K.xi = mu |xi|^2 I + (lambda + mu) xi xi  -> inverse in closed form
    lam, mu = 2.0, 1.5
    K4 = cubic_stiffness(lam + 2 * mu, lam, mu)
    g = Grid((4, 4, 4), 1.0)
    Ainv = g.acoustic_inverse(K4)
    k = g.xit[1, 2, 3]
    k2 = k @ k
    exact = (np.eye(3) - (lam + mu) / (lam + 2 * mu) * np.outer(k, k) / k2) / (mu * k2)
    assert np.allclose(Ainv[1, 2, 3], exact, rtol=1e-14, atol=0)
    assert np.all(Ainv[0, 0, 0] == 0)
    assert to_mandel4(K4).shape == (6, 6)
