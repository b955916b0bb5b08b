"""Pins of the oracle's momentum solver (Sec. 3.1, eqs. momentum, fdef, newton, precf):
homogeneous medium, the two-phase laminate closed form, equilibrium and macro control."""
import numpy as np

from oracle import Grid, solve_mechanics, cubic_stiffness, to_mandel2, to_mandel4, from_mandel2
from oracle.increment import tensor6


def _elastic(Cm):
    """Linear elastic 'constitutive update' with per-voxel Mandel stiffness Cm (M,6,6)."""
    def constit(e):
        sig = np.einsum("mij,mj->mi", Cm, e)
        w = 0.5 * np.einsum("mi,mi->m", sig, e)
        return sig, np.zeros((len(e), 12)), Cm.copy(), w
    return constit


def _iso(lam, mu):
    return to_mandel4(cubic_stiffness(lam + 2 * mu, lam, mu))


def test_homogeneous_medium_needs_one_krylov_iteration():
    rng = np.random.default_rng(0)
    n = (8, 6, 4)
    g = Grid(n, 1e-6)
    M = g.M
    Cm = np.broadcast_to(to_mandel4(cubic_stiffness(168.4e9, 121.4e9, 75.4e9)), (M, 6, 6)).copy()
    ebar = np.array([[1e-3, 2e-4, 0], [2e-4, -5e-4, 1e-4], [0, 1e-4, 3e-4]])
    u = rng.standard_normal(n + (3,)) * 1e-9
    fluct = g.to_flat(g.ifft(g.sym_grad_hat(g.fft(u))))
    eps0 = ebar[None] + fluct
    stats = {}
    eps, sig, _ = solve_mechanics(g, eps0, np.zeros((M, 3, 3)), np.ones(M), _elastic(Cm),
                                  1e-12, 1e-12, 10, 100, stats)
    assert np.abs(eps - ebar[None]).max() <= 1e-14 * np.abs(ebar).max()
    assert stats["matvecs"] <= 2 and stats["newton"] <= 2
    ref = from_mandel2(Cm[0] @ to_mandel2(ebar))
    assert np.abs(from_mandel2(sig) - ref[None]).max() <= 1e-12 * np.abs(ref).max()


def _laminate_closed_form(ebar, C1, C2, f1):
    """Layers normal to e1: eps_p = ebar + sym(a_p (x) e1), traction continuity, f1 a1 + f2 a2 = 0."""
    C1t = np.asarray(C1)
    C2t = np.asarray(C2)
    e1 = np.array([1.0, 0, 0])

    def jump_op(C):   # a -> (C : sym(a (x) e1)) . e1
        A = np.zeros((3, 3))
        for k in range(3):
            a = np.zeros(3); a[k] = 1
            E = 0.5 * (np.outer(a, e1) + np.outer(e1, a))
            A[:, k] = np.einsum("ijkl,kl->ij", C, E) @ e1
        return A
    f2 = 1 - f1
    # a2 = -f1/f2 a1 ; (C1:(ebar+E(a1)) - C2:(ebar+E(a2))).e1 = 0
    lhs = jump_op(C1t) + f1 / f2 * jump_op(C2t)
    rhs = -(np.einsum("ijkl,kl->ij", C1t - C2t, ebar) @ e1)
    a1 = np.linalg.solve(lhs, rhs)
    a2 = -f1 / f2 * a1
    E = lambda a: ebar + 0.5 * (np.outer(a, e1) + np.outer(e1, a))
    return E(a1), E(a2)


def test_two_phase_laminate_closed_form():
    n = (8, 4, 4)
    g = Grid(n, 1.0)
    i = np.arange(n[0])
    phase1 = (i < 4)                                  # even layer widths (Nyquist reading)
    ph = g.to_flat(np.broadcast_to(phase1[:, None, None], n).astype(float)) > 0.5
    Ca = cubic_stiffness(3.0 + 2 * 1.0, 3.0, 1.0)     # lambda 3, mu 1
    Cb = cubic_stiffness(1.0 + 2 * 5.0, 1.0, 5.0)     # contrast 5 in shear
    Cm = np.where(ph[:, None, None], to_mandel4(Ca)[None], to_mandel4(Cb)[None])
    ebar = np.array([[1e-3, 3e-4, -2e-4], [3e-4, 5e-4, 1e-4], [-2e-4, 1e-4, -4e-4]])
    M = g.M
    eps, _, _ = solve_mechanics(g, np.broadcast_to(ebar, (M, 3, 3)).copy(), np.zeros((M, 3, 3)),
                                np.ones(M), _elastic(Cm), 1e-13, 1e-14, 20, 500)
    ea, eb = _laminate_closed_form(ebar, Ca, Cb, 0.5)
    assert np.abs(eps[ph] - ea).max() <= 1e-13
    assert np.abs(eps[~ph] - eb).max() <= 1e-13
    assert np.abs(eps.mean(0) - ebar).max() <= 1e-16 + 1e-14 * np.abs(ebar).max()


def test_equilibrium_divergence_vanishes_and_macro_strain_is_imposed():
    rng = np.random.default_rng(5)
    n = (6, 6, 6)
    g = Grid(n, 1e-6)
    M = g.M
    # random isotropic phases (contrast ~10) and a degradation field
    mu = np.exp(rng.uniform(0, np.log(10), M)) * 1e10
    Cm = np.array([_iso(2 * m, m) for m in mu])
    gphi = rng.uniform(0.1, 1.0, M)
    ebar = np.diag([0.0, 2e-3, 0.0])
    eps, sig, _ = solve_mechanics(g, np.broadcast_to(ebar, (M, 3, 3)).copy(), np.zeros((M, 3, 3)),
                                  gphi, _elastic(Cm), 1e-12, 1e-12, 20, 2000)
    s = g.to_grid(gphi[:, None, None] * from_mandel2(sig))
    sh = g.fft(s)
    div = np.abs(g.div_hat(sh)).max()
    assert div <= 1e-9 * np.abs(sh).max() * np.abs(g.xit).max()
    assert np.abs(tensor6(eps).mean(0) - tensor6(ebar[None])[0]).max() <= 1e-17
