"""Pins of the oracle's rotated-scheme discrete derivative (the discrete derivative remedy
that Sec. 3.1 names against Gibbs oscillations): the Fourier symbol against the
real-space stencil (forward difference averaged over the four parallel voxel edges), the
discrete integration by parts, the null space, the two-phase laminate closed form (exact
for this stencil with layers of any width) and a polycrystal increment."""
import numpy as np

from oracle import Grid, solve_mechanics, cubic_stiffness, to_mandel2, to_mandel4, OracleRVE
from synth import small_polycrystal, make_inputs
from test_oracle_mechanics import _elastic, _laminate_closed_form


def _stencil_strain(u, h):
    """Rotated-scheme strain of a periodic displacement grid u (N1,N2,N3,3), brute force."""
    def fwd(f, a):                           # forward difference along a
        return (np.roll(f, -1, axis=a) - f) / h

    def avg(f, a):                           # average with the neighbour along a
        return 0.5 * (f + np.roll(f, -1, axis=a))
    G = np.zeros(u.shape[:3] + (3, 3))
    for a in range(3):
        others = [b for b in range(3) if b != a]
        for j in range(3):
            d = fwd(u[..., j], a)
            for b in others:
                d = avg(d, b)
            G[..., a, j] = d                 # derivative along a of u_j
    return 0.5 * (G + np.swapaxes(G, -1, -2))


def test_symbol_matches_real_space_stencil():
    rng = np.random.default_rng(0)
    for n in [(6, 4, 5), (8, 8, 8), (3, 6, 2)]:
        g = Grid(n, 0.7, scheme=1)
        u = rng.standard_normal(n + (3,))
        e_fft = g.ifft(g.sym_grad_hat(g.fft(u)))
        e_ref = _stencil_strain(u, 0.7)
        assert np.abs(e_fft - e_ref).max() <= 1e-13 * np.abs(e_ref).max()


def test_discrete_integration_by_parts_and_null_space():
    rng = np.random.default_rng(1)
    n = (6, 4, 8)
    g = Grid(n, 1.3, scheme=1)
    u = rng.standard_normal(n + (3,))
    s = rng.standard_normal(n + (3, 3))
    s = 0.5 * (s + np.swapaxes(s, -1, -2))
    lhs = (g.ifft(g.sym_grad_hat(g.fft(u))) * s).sum()
    rhs = -(u * g.ifft(g.div_hat(g.fft(s)))).sum()          # <eps(u), s> = -<u, div s>
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the symbol vanishes at zero frequency and on the lines with two Nyquist indices
    k = g.k
    assert np.abs(k[0, 0, 0]).max() == 0.0
    assert np.abs(k[3, 2, :]).max() == 0.0 and np.abs(k[3, :, 4]).max() == 0.0
    assert np.abs(k[:, 2, 4]).max() == 0.0
    # elsewhere it does not (the acoustic tensor is invertible there): the three lines
    # share one point, so the zero set has 1 + (n3 + n2 + n1 - 2) members
    assert g.nonzero.sum() == g.M - 1 - (n[2] + n[1] + n[0] - 2)


def test_two_phase_laminate_closed_form_any_layer_width():
    n = (9, 4, 4)
    g = Grid(n, 1.0, scheme=1)
    i = np.arange(n[0])
    ph = g.to_flat(np.broadcast_to((i < 4)[:, None, None], n).astype(float)) > 0.5
    Ca = cubic_stiffness(3.0 + 2 * 1.0, 3.0, 1.0)
    Cb = cubic_stiffness(1.0 + 2 * 5.0, 1.0, 5.0)
    Cm = np.where(ph[:, None, None], to_mandel4(Ca)[None], to_mandel4(Cb)[None])
    ebar = np.array([[1e-3, 3e-4, -2e-4], [3e-4, 5e-4, 1e-4], [-2e-4, 1e-4, -4e-4]])
    M = g.M
    eps, _, _ = solve_mechanics(g, np.broadcast_to(ebar, (M, 3, 3)).copy(), np.zeros((M, 3, 3)),
                                np.ones(M), _elastic(Cm), 1e-13, 1e-14, 20, 500)
    ea, eb = _laminate_closed_form(ebar, Ca, Cb, 4.0 / 9.0)
    assert np.abs(eps[ph] - ea).max() <= 1e-15
    assert np.abs(eps[~ph] - eb).max() <= 1e-15


def test_polycrystal_increment_is_equilibrated_for_the_rotated_divergence():
    w = small_polycrystal(n=8, n_grains=4, seed=5, amplitude=0.008).parity()
    d = dict(w.desc(), scheme=1)
    inp = make_inputs(w)
    o = OracleRVE(d, inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(3):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k])
    g = o.grid
    from oracle.increment import from_tensor6
    f = o.fields()
    sh = g.fft(g.to_grid(from_tensor6(f["stress"])))
    div = np.abs(g.div_hat(sh)).max() / (np.abs(sh).max() * np.abs(g.k).max())
    assert div <= 1e-12
    assert abs(f["strain"].mean(0)[1] - sum(inp["deps"][:3])) <= 1e-15
    # the spectral divergence of the same field does not vanish (a different discrete
    # equilibrium)
    gs = Grid(w.n, w.h)
    assert np.abs(gs.div_hat(sh)).max() / (np.abs(sh).max() * np.abs(gs.xit).max()) > 1e-6
