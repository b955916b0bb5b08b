"""Pins of the oracle's mixed (strain/stress) macroscopic control (the DBFFT mixed extension
the paper relies on, Sec. 3.1): a homogeneous anisotropic medium in closed form (uniaxial
stress and pure stress control), the two-phase laminate whose effective stiffness is
known in closed form, and stress-free lateral components in a yielding polycrystal."""
import numpy as np

from oracle import (Grid, solve_mechanics, cubic_stiffness, rotate4, quat_to_rot, to_mandel2,
                    to_mandel4, from_mandel2, OracleRVE)
from oracle.increment import tensor6, from_tensor6
from synth import shoemake_quaternions, small_polycrystal, make_inputs
from test_oracle_mechanics import _elastic, _laminate_closed_form

UNIAXIAL_Y = [0, 2, 3, 4, 5]              # Mandel indices with zero macro stress


def _solve(g, Cm, E0, free, tgt):
    M = g.M
    eps0 = np.broadcast_to(from_mandel2(E0[None])[0], (M, 3, 3)).copy()
    return solve_mechanics(g, eps0, np.zeros((M, 3, 3)), np.ones(M), _elastic(Cm), 1e-13, 1e-14,
                           20, 500, free=free, sig_target=tgt)


def test_homogeneous_anisotropic_medium_under_uniaxial_and_pure_stress():
    R = quat_to_rot(shoemake_quaternions(1, np.random.default_rng(2)))[0]
    C = to_mandel4(rotate4(cubic_stiffness(168.4e9, 121.4e9, 75.4e9), R))
    g = Grid((6, 4, 4), 1e-6)
    Cm = np.broadcast_to(C, (g.M, 6, 6)).copy()
    # uniaxial stress along y: E_yy = 1e-3, every other macro stress 0
    E0 = np.zeros(6); E0[1] = 1e-3
    eps, sig, _ = _solve(g, Cm, E0, UNIAXIAL_Y, np.zeros(6))
    F, P = UNIAXIAL_Y, [1]
    Ef = -np.linalg.solve(C[np.ix_(F, F)], C[np.ix_(F, P)] @ E0[P])
    E = E0.copy(); E[F] = Ef
    assert np.abs(to_mandel2(eps) - E[None]).max() <= 1e-13 * 1e-3
    assert np.abs(sig[:, F]).max() <= 1e-12 * np.abs(sig[:, 1]).max()
    # pure stress control: E = C^-1 sigma
    S = np.array([3e8, -1e8, 5e7, 2e7, -4e7, 1e8])
    eps, sig, _ = _solve(g, Cm, np.zeros(6), list(range(6)), S)
    assert np.abs(to_mandel2(eps) - np.linalg.solve(C, S)[None]).max() <= 1e-13 * 1e-3
    assert np.abs(sig - S[None]).max() <= 1e-12 * np.abs(S).max()


def test_two_phase_laminate_under_mixed_control():
    n = (8, 4, 4)
    g = Grid(n, 1.0)
    i = np.arange(n[0])
    ph = g.to_flat(np.broadcast_to((i < 4)[:, None, None], n).astype(float)) > 0.5
    Ca = cubic_stiffness(3.0 + 2 * 1.0, 3.0, 1.0)
    Cb = cubic_stiffness(1.0 + 2 * 5.0, 1.0, 5.0)
    Cm = np.where(ph[:, None, None], to_mandel4(Ca)[None], to_mandel4(Cb)[None])
    # effective stiffness of the laminate, column by column from the closed form
    Ceff = np.zeros((6, 6))
    for b in range(6):
        e = np.zeros(6); e[b] = 1.0
        ea, eb = _laminate_closed_form(from_mandel2(e[None])[0], Ca, Cb, 0.5)
        sa = np.einsum("ijkl,kl->ij", Ca, ea)
        sb = np.einsum("ijkl,kl->ij", Cb, eb)
        Ceff[:, b] = to_mandel2((0.5 * (sa + sb))[None])[0]
    F, P = UNIAXIAL_Y, [1]
    E = np.zeros(6); E[1] = 1e-3
    E[F] = -np.linalg.solve(Ceff[np.ix_(F, F)], Ceff[np.ix_(F, P)] @ E[P])
    ea, eb = _laminate_closed_form(from_mandel2(E[None])[0], Ca, Cb, 0.5)
    E0 = np.zeros(6); E0[1] = 1e-3
    eps, sig, _ = _solve(g, Cm, E0, F, np.zeros(6))
    assert np.abs(eps[ph] - ea).max() <= 1e-15
    assert np.abs(eps[~ph] - eb).max() <= 1e-15
    assert np.abs(sig.mean(0)[F]).max() <= 1e-12 * np.abs(sig.mean(0)[1])


def test_yielding_polycrystal_keeps_the_lateral_macro_stress_at_zero():
    w = small_polycrystal(n=8, n_grains=4, seed=5, amplitude=0.008).parity()
    inp = make_inputs(w)
    o = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    mask = 0b111101                                 # all but yy under stress control
    eyy = 0.0
    for k in range(5):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), mask)
        eyy += inp["deps"][k]
        ms, me = st["macro_stress"], st["macro_strain"]
        assert abs(me[1] - eyy) <= 1e-15
        assert np.abs(ms[[0, 2, 3, 4, 5]]).max() <= 1e-9 * abs(ms[1])
    assert np.abs(o.epsp).max() > 1e-4                 # yielded
    assert me[0] < 0 and me[2] < 0                     # lateral contraction
