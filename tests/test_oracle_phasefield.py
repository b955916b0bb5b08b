"""Pins of the oracle's phase-field parts (eqs. strpf, phase, decMiehe, precph) and of the
Nye-tensor GND density (eq. nye1, Fourier curl, regularisation)."""
import numpy as np

from oracle import (Grid, split_positive, solve_phase_field, nye_tensor, gnd_density,
                    gnd_matrix, quat_to_rot, fcc_slip_systems)
from synth import shoemake_quaternions


def test_uniform_driving_state_closed_form():
    g = Grid((4, 6, 8), 1e-6)
    S = np.full(g.M, 0.7)
    phi = solve_phase_field(g, S, 2e-6, rtol=1e-14)
    assert np.abs(phi - 1.4 / 2.4).max() <= 1e-14


def test_zero_driving_state_gives_zero():
    g = Grid((4, 4, 4), 1.0)
    assert np.all(solve_phase_field(g, np.zeros(g.M), 2.0) == 0)


def test_at2_profile_exact_discrete_and_physical():
    # a single driven plane x = 0: away from it phi solves (1 - l^2 lap) phi = 0, so
    # phi_j / phi_0 = G_j / G_0 with G the periodic Green function of 1 + l^2 xi^2
    h = 1.0
    for ell in (2.0, 8.0):
        N = int(32 * ell)                 # images of the periodic cell decay out of the band
        g = Grid((N, 2, 2), h)
        S = np.zeros((N, 2, 2))
        S[0] = 50.0
        phi = g.to_grid(solve_phase_field(g, g.to_flat(S), ell, rtol=1e-15))[:, 0, 0]
        xi = 2 * np.pi * np.fft.fftfreq(N, 1.0 / N) / (N * h)
        G = np.fft.ifft(1.0 / (1.0 + ell ** 2 * xi ** 2)).real
        assert np.abs(phi / phi[0] - G / G[0]).max() <= 1e-12
        x = np.minimum(np.arange(N), N - np.arange(N)) * h
        near = x <= 3 * ell
        dev = np.abs(phi / phi[0] - np.exp(-x / ell))[near].max()
        assert dev <= (0.09 if ell == 2.0 else 0.03)
        band = (x >= ell) & (x <= 4 * ell) & (np.arange(N) < N // 2)
        ratios = phi[1:][band[1:]] / phi[:-1][band[1:]]
        assert np.all(np.abs(ratios / np.exp(-h / ell) - 1) <= 0.035)


def test_spectral_split_properties():
    rng = np.random.default_rng(0)
    E = rng.standard_normal((50, 3, 3)); E = E + np.swapaxes(E, 1, 2)
    Ep = split_positive(E)
    En = -split_positive(-E)
    assert np.abs(Ep + En - E).max() <= 1e-14 * 10
    A = rng.standard_normal((5, 3, 3))
    PD = np.einsum("mij,mkj->mik", A, A) + 0.1 * np.eye(3)
    assert np.abs(split_positive(PD) - PD).max() <= 1e-14 * np.abs(PD).max() * 10
    assert np.abs(split_positive(-PD)).max() == 0
    # repeated eigenvalues: diag(1, 1, -2) rotated
    Q = quat_to_rot(shoemake_quaternions(1, rng))[0]
    D = Q @ np.diag([1.0, 1.0, -2.0]) @ Q.T
    assert np.abs(split_positive(D[None])[0] - Q @ np.diag([1.0, 1, 0]) @ Q.T).max() < 1e-14


def test_gnd_matrix_rank_and_pseudoinverse():
    A = gnd_matrix()
    assert A.shape == (9, 18) and np.linalg.matrix_rank(A) == 9
    # minimum-norm solution: A A^+ = I and ||A^+ v||^2 = v^T (A A^T)^-1 v
    Ap = np.linalg.pinv(A)
    assert np.allclose(A @ Ap, np.eye(9), atol=1e-13)
    v = np.random.default_rng(1).standard_normal(9)
    assert np.isclose(np.linalg.norm(Ap @ v) ** 2, v @ np.linalg.solve(A @ A.T, v))


def test_nye_of_gradient_and_uniform_fields_vanish():
    rng = np.random.default_rng(2)
    n = (8, 6, 4)
    g = Grid(n, 1e-6)
    v = rng.standard_normal(n + (3,))
    vh = g.fft(v)
    beta = g.to_flat(g.ifft(1j * vh[..., :, None] * g.xit[..., None, :]))   # d_l v_i
    lam = nye_tensor(g, beta, 2e-6)
    assert np.abs(lam).max() <= 1e-12 * np.abs(beta).max() / 1e-6
    lam_u = nye_tensor(g, np.broadcast_to(rng.standard_normal((3, 3)), (g.M, 3, 3)), 2e-6)
    assert np.abs(lam_u).max() <= 1e-9


def test_nye_single_mode_closed_form():
    # beta = gamma(x) s (x) n with gamma = A sin(2 pi x / L): Lambda_ij = s_i (grad gamma x n)_j
    n, h, A = (16, 2, 2), 1e-6, 1e-3
    g = Grid(n, h)
    L = n[0] * h
    s, nn = fcc_slip_systems()
    s, nn = s[3], nn[3]
    x = (np.arange(n[0]) + 0.5) * h
    gam = A * np.sin(2 * np.pi * x / L)
    beta = g.to_flat(np.broadcast_to((gam[:, None, None] * np.outer(s, nn)[None])[:, None, None],
                                     n + (3, 3)).copy())
    ell_fp = 1.5e-6
    lam = g.to_grid(nye_tensor(g, beta, ell_fp))[:, 0, 0]
    k = 2 * np.pi / L
    dgam = A * k * np.cos(k * x) / (1 + ell_fp ** 2 * k ** 2)    # regularised derivative
    exact = dgam[:, None, None] * np.outer(s, np.cross([1.0, 0, 0], nn))[None]
    assert np.abs(lam - exact).max() <= 1e-12 * np.abs(exact).max()


def test_gnd_density_is_frame_independent():
    rng = np.random.default_rng(3)
    R = quat_to_rot(shoemake_quaternions(4, rng))
    lam_c = rng.standard_normal((4, 3, 3)) * 1e3
    lam_s = np.einsum("mia,mab,mjb->mij", R, lam_c, R)       # sample frame
    rho = gnd_density(lam_s, R, 3.5e-10)
    A = gnd_matrix()
    ref = np.sqrt(np.einsum("mi,ij,mj->m", lam_c.reshape(4, 9),
                            np.linalg.inv(A @ A.T), lam_c.reshape(4, 9))) / 3.5e-10
    assert np.allclose(rho, ref, rtol=1e-12)


def test_dirichlet_phase_field_against_dense_solve_and_point_green_function():
    """Pre-set crack voxels held at phi = 1 (Dirichlet option): brute force on a small grid
    (the operator assembled column by column, the free block solved densely), the point
    condition closed form phi = G(x - x0) / G(0) with G the discrete Green function of
    1 - l^2 lap (S = 0), and no fixed voxel reducing to the free solve."""
    from oracle import Grid, solve_phase_field, solve_phase_field_dirichlet
    g = Grid((8, 4, 3), 1.0)
    ell = 1.3
    M = g.M
    rng = np.random.default_rng(4)
    S = rng.uniform(0.0, 2.0, M)
    fixed = np.zeros(M, dtype=bool)
    fixed[[3, 17, 40]] = True
    # dense operator A = (1 + 2S) - l^2 lap on flat vectors
    A = np.zeros((M, M))
    for j in range(M):
        e = np.zeros(M); e[j] = 1.0
        lap = g.to_flat(g.ifft(ell ** 2 * g.xi2 * g.fft(g.to_grid(e))))
        A[:, j] = (1.0 + 2.0 * S) * e + lap
    F = ~fixed
    phi_ref = np.ones(M)
    phi_ref[F] = np.linalg.solve(A[np.ix_(F, F)], 2.0 * S[F] - A[np.ix_(F, fixed)] @ np.ones(3))
    phi = solve_phase_field_dirichlet(g, S, ell, fixed, rtol=1e-14)
    assert np.abs(phi - phi_ref).max() <= 1e-12
    # point condition, S = 0
    one = np.zeros(M, dtype=bool); one[21] = True
    phi = solve_phase_field_dirichlet(g, np.zeros(M), ell, one, rtol=1e-14)
    delta = np.zeros(M); delta[21] = 1.0
    G = g.to_flat(g.ifft(g.fft(g.to_grid(delta)) / (1.0 + ell ** 2 * g.xi2)))
    assert np.abs(phi - G / G[21]).max() <= 1e-12
    # no fixed voxel: the free solve
    a = solve_phase_field_dirichlet(g, S, ell, np.zeros(M, dtype=bool), rtol=1e-14)
    b = solve_phase_field(g, S, ell, rtol=1e-14)
    assert np.abs(a - b).max() <= 1e-12


def test_dirichlet_phase_field_degenerate_sets():
    """Every voxel fixed: nothing to solve, phi = 1; a single free voxel: the scalar balance
    (1 + 2S + l^2 lap_0) u = 2S - (1 + 2S) * 0 - l^2 (lap 1_fixed)_0 written out by hand."""
    from oracle import Grid, solve_phase_field_dirichlet
    g = Grid((4, 4, 2), 1.0)
    M = g.M
    S = np.linspace(0.0, 1.0, M)
    phi = solve_phase_field_dirichlet(g, S, 0.7, np.ones(M, dtype=bool), rtol=1e-14)
    assert np.all(phi == 1.0)
    fixed = np.ones(M, dtype=bool)
    fixed[5] = False
    ell = 0.7
    phi = solve_phase_field_dirichlet(g, S, ell, fixed, rtol=1e-14)
    # diagonal of -l^2 lap (spectral): l^2 mean(|xi|^2); its action on 1_fixed at voxel 5:
    # -l^2 lap 1 = 0 for the constant field, so -l^2 lap 1_fixed = l^2 lap e_5 = -diag e_5
    d = ell ** 2 * g.xi2.mean()
    u = (2.0 * S[5] + d) / (1.0 + 2.0 * S[5] + d)
    assert abs(phi[5] - u) <= 1e-12
    assert np.all(phi[fixed] == 1.0)
