"""Pins of the oracle's pointwise plane stress for plates one voxel thick (Sec. 4.1-4.3):
the reduced stiffness of a homogeneous anisotropic plate (the inverse of the in-plane
block of the compliance, a textbook identity independent of the condensation the oracle
uses), the two-phase plate laminate in closed form under strain and under uniaxial
control, the condensed tangent against finite differences of the constrained stress, a
yielding homogeneous plate against the three-dimensional oracle under uniaxial stress,
and the invariants of a yielding polycrystal plate (zero out-of-plane stress at every
voxel, in-plane equilibrium and compatibility, stress-free lateral macro components)."""
import numpy as np
import pytest

from oracle import (Grid, GrainTables, OracleRVE, PowerLaw, cubic_stiffness, rotate4,
                    quat_to_rot, return_map, to_mandel2, to_mandel4, from_mandel2)
from oracle.planestress import (P_IDX, O_IDX, local_plane_stress, condensed_tangent,
                                solve_mechanics_plane)
from synth import shoemake_quaternions, small_polycrystal, make_inputs
from test_oracle_mechanics import _elastic

C11, C12, C44 = 168.4e9, 121.4e9, 75.4e9
UNIAXIAL_PLATE = [0, 5]          # Mandel xx, xy stress free; yy strain controlled


def _crystal(seed):
    R = quat_to_rot(shoemake_quaternions(1, np.random.default_rng(seed)))[0]
    return to_mandel4(rotate4(cubic_stiffness(C11, C12, C44), R))


def _reduced(C):
    """Plane-stress stiffness (in-plane Mandel order xx, yy, xy): the inverse of the
    in-plane block of the compliance S = C^-1."""
    S = np.linalg.inv(C)
    return np.linalg.inv(S[np.ix_(P_IDX, P_IDX)]), S


def _solve(g, Cm, EP, free=(), tgt=None, stats=None):
    M = g.M
    E6 = np.zeros(6)
    E6[P_IDX] = EP
    eps0 = np.broadcast_to(from_mandel2(E6[None])[0], (M, 3, 3)).copy()
    return solve_mechanics_plane(g, eps0, np.zeros((M, 3, 3)), np.ones(M), _elastic(Cm), 1e-13,
                                 1e-14, 20, 500, stats=stats, free=free, sig_target=tgt)


def test_homogeneous_anisotropic_plate_has_the_reduced_stiffness():
    C = _crystal(2)
    Q, S = _reduced(C)
    g = Grid((6, 4, 1), 1e-6)
    Cm = np.broadcast_to(C, (g.M, 6, 6)).copy()
    EP = np.array([1.0e-3, -4e-4, 3e-4 * np.sqrt(2)])
    st = {}
    eps, sig, _ = _solve(g, Cm, EP, stats=st)
    sP = Q @ EP
    assert np.abs(sig[:, P_IDX] - sP[None]).max() <= 1e-12 * np.abs(sP).max()
    assert np.abs(sig[:, O_IDX]).max() <= 1e-12 * np.abs(sP).max()
    eO = S[np.ix_(O_IDX, P_IDX)] @ sP                 # out-of-plane strain of the free plate
    em = to_mandel2(eps)
    assert np.abs(em[:, O_IDX] - eO[None]).max() <= 1e-13 * np.abs(EP).max()
    assert np.abs(em[:, P_IDX] - EP[None]).max() <= 1e-15
    assert st["newton"] == 1                          # the uniform start is the solution
    # uniaxial control along y: sigma_yy = E_yy / S_yy,yy, every other stress zero
    E0 = np.array([0.0, 1e-3, 0.0])
    eps, sig, _ = _solve(g, Cm, E0, free=UNIAXIAL_PLATE, tgt=np.zeros(6))
    syy = 1e-3 / S[1, 1]
    assert np.abs(sig[:, 1] - syy).max() <= 1e-12 * abs(syy)
    assert np.abs(np.delete(sig, 1, axis=1)).max() <= 1e-12 * abs(syy)
    assert np.abs(to_mandel2(eps) - (S[:, 1] * syy)[None]).max() <= 1e-13 * 1e-3
    # pure in-plane stress control: eps = S sigma with sigma_O = 0
    T = np.zeros(6)
    T[P_IDX] = [3e8, -1e8, 1e8 * np.sqrt(2)]
    eps, sig, _ = _solve(g, Cm, np.zeros(3), free=[0, 1, 5], tgt=T)
    assert np.abs(sig - T[None]).max() <= 1e-12 * np.abs(T).max()
    assert np.abs(to_mandel2(eps) - (S @ T)[None]).max() <= 1e-13 * 1e-3


def _plate_laminate(Ca, Cb, f, EP=None, uniaxial_eyy=None):
    """Layers normal to x, uniform fields per phase: eps_yy continuous, sigma_xx and
    sigma_xy continuous, volume averages equal to the macro values.  Returns the
    in-plane Mandel strains and stresses of both phases."""
    Qa, _ = _reduced(Ca)
    Qb, _ = _reduced(Cb)
    if uniaxial_eyy is not None:                    # sigma_xx = sigma_xy = 0 everywhere
        out = []
        for C in (Ca, Cb):
            S = np.linalg.inv(C)
            syy = uniaxial_eyy / S[1, 1]
            out.append((S[np.ix_(P_IDX, P_IDX)][:, 1] * syy, np.array([0.0, syy, 0.0])))
        return out
    A = np.zeros((6, 6))
    b = np.zeros(6)
    A[0, 1], A[0, 4] = 1.0, -1.0                              # eps_yy^a = eps_yy^b
    for r, c in enumerate((0, 1, 2)):                         # f eps^a + (1-f) eps^b = E
        A[1 + r, c], A[1 + r, 3 + c] = f, 1.0 - f
        b[1 + r] = EP[c]
    for r, c in enumerate((0, 2)):                            # traction continuity
        A[4 + r, 0:3], A[4 + r, 3:6] = Qa[c], -Qb[c]
    x = np.linalg.solve(A, b)
    return [(x[0:3], Qa @ x[0:3]), (x[3:6], Qb @ x[3:6])]


@pytest.mark.parametrize("uniaxial", [False, True])
def test_two_phase_plate_laminate_closed_form(uniaxial):
    n = (8, 4, 1)
    g = Grid(n, 1.0)
    i = np.arange(n[0])
    # an even number of layers per phase: the phase indicator then has no Nyquist
    # component, which the compatible fields of the spectral gradient cannot carry
    ph = g.to_flat(np.broadcast_to((i < 6)[:, None, None], n).astype(float)) > 0.5
    Ca, Cb = _crystal(5), 0.4 * _crystal(6)
    Cm = np.where(ph[:, None, None], Ca[None], Cb[None])
    f = 6.0 / 8.0
    if uniaxial:
        ref = _plate_laminate(Ca, Cb, f, uniaxial_eyy=1e-3)
        eps, sig, _ = _solve(g, Cm, np.array([0.0, 1e-3, 0.0]), free=UNIAXIAL_PLATE,
                             tgt=np.zeros(6))
    else:
        EP = np.array([1.0e-3, -4e-4, 3e-4 * np.sqrt(2)])
        ref = _plate_laminate(Ca, Cb, f, EP=EP)
        st = {}
        eps, sig, _ = _solve(g, Cm, EP, stats=st)
        assert st["newton"] == 2                      # linear: the first step is exact
    em = to_mandel2(eps)
    for mask, C, (eP, sP) in ((ph, Ca, ref[0]), (~ph, Cb, ref[1])):
        scale = np.abs(sP).max()
        assert np.abs(em[mask][:, P_IDX] - eP[None]).max() <= 1e-14
        assert np.abs(sig[mask][:, P_IDX] - sP[None]).max() <= 1e-12 * scale
        assert np.abs(sig[mask][:, O_IDX]).max() <= 1e-12 * scale
        eO = np.linalg.inv(C)[np.ix_(O_IDX, P_IDX)] @ sP
        assert np.abs(em[mask][:, O_IDX] - eO[None]).max() <= 1e-14


def test_condensed_tangent_is_the_derivative_of_the_constrained_stress():
    t = GrainTables(shoemake_quaternions(1, np.random.default_rng(12)), C11, C12, C44)
    law = PowerLaw(1e-3, 20.0)
    g = np.array([50e6])
    constit = lambda e: return_map(e, np.zeros((1, 6)), g, 1.0, t.C, t.S, t.P, law=law)
    EP = np.array([1.5e-3, -2e-4, 4e-4 * np.sqrt(2)])
    e0 = np.zeros((1, 6))
    e0[0, P_IDX] = EP
    e, sig, dgam, K, _ = local_plane_stress(constit, e0)
    assert np.abs(dgam).max() > 1e-5                   # on the plastic branch
    Kc = condensed_tangent(K)[0]
    fd = np.zeros((3, 3))
    h = 1e-8
    for j in range(3):
        col = []
        for s in (1.0, -1.0):
            ej = e.copy()
            ej[0, P_IDX[j]] += s * h
            col.append(local_plane_stress(constit, ej)[1][0, P_IDX])
        fd[:, j] = (col[0] - col[1]) / (2 * h)
    assert np.abs(fd - Kc).max() <= 1e-5 * np.abs(Kc).max()
    # the unconstrained in-plane block is stiffer: the condensation is not a no-op
    assert np.abs(K[0][np.ix_(P_IDX, P_IDX)] - Kc).max() > 1e-2 * np.abs(Kc).max()


def test_yielding_homogeneous_plate_matches_uniaxial_stress_in_3d():
    w = small_polycrystal(n=(4, 3, 1), n_grains=1, seed=8, amplitude=0.008).parity()
    inp = make_inputs(w)
    plate = OracleRVE(dict(w.desc(), plane_stress=1), inp["grain"], inp["quat"],
                      inp["tau_c0"], inp["phi0"])
    solid = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(6):
        sp = plate.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), 0b100001)
        ss = solid.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), 0b111101)
        scale = np.abs(ss["macro_stress"]).max()
        assert np.abs(sp["macro_stress"] - ss["macro_stress"]).max() <= 1e-11 * scale
        assert np.abs(plate.eps - solid.eps).max() <= 1e-12 * np.abs(solid.eps).max()
    assert plate.Wp.max() > 1e4 and np.abs(plate.Wp - solid.Wp).max() <= 1e-10 * solid.Wp.max()
    assert np.abs(plate.Gs - solid.Gs).max() <= 1e-10 * solid.Gs.max()


def test_yielding_polycrystal_plate_invariants():
    w = small_polycrystal(n=(12, 10, 1), n_grains=5, seed=3, amplitude=0.008).parity()
    inp = make_inputs(w)
    o = OracleRVE(dict(w.desc(), plane_stress=1), inp["grain"], inp["quat"], inp["tau_c0"],
                  inp["phi0"])
    for k in range(5):
        st = o.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), 0b100001)
    g = o.grid
    scale = np.abs(o.sig).max()
    assert o.Wp.max() > 1e4
    assert np.abs(o.sig[:, O_IDX]).max() <= 1e-12 * scale           # pointwise plane stress
    ms = st["macro_stress"]
    assert max(abs(ms[0]), abs(ms[5])) <= 1e-10 * abs(ms[1])        # uniaxial along y
    # in-plane equilibrium: i xi~ . F{g sigma} = 0 on every frequency (x, y rows)
    gphi = o.degradation(o.phi)
    sh = g.fft(g.to_grid(gphi[:, None, None] * from_mandel2(o.sig)))
    div = np.abs(g.div_hat(sh)[..., :2]).max()
    assert div <= 1e-11 * np.abs(g.xit).max() * np.abs(sh).max()
    # in-plane compatibility: xi_y^2 e_xx + xi_x^2 e_yy - 2 xi_x xi_y e_xy = 0
    eh = g.fft(g.to_grid(o.eps))
    kx, ky = g.xit[..., 0], g.xit[..., 1]
    sv = ky ** 2 * eh[..., 0, 0] + kx ** 2 * eh[..., 1, 1] - 2 * kx * ky * eh[..., 0, 1]
    assert np.abs(sv).max() <= 1e-13 * np.abs(g.xit).max() ** 2 * np.abs(eh[..., :2, :2]).max()
    # the out-of-plane strain is a local field, not a displacement gradient
    ezz = o.eps[:, 2, 2]
    assert ezz.max() - ezz.min() > 1e-2 * np.abs(ezz).max()
    # a periodic slab without the condition keeps sigma_zz inside the grains
    s3 = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    for k in range(5):
        s3.step([0, inp["deps"][k], 0, 0, 0, 0], inp["dt"][k], np.zeros(6), 0b111101)
    assert np.abs(s3.sig[:, 2]).max() > 1e-2 * np.abs(s3.sig).max()


def test_plane_stress_options_are_validated():
    w = small_polycrystal(n=(4, 4, 2), n_grains=2, seed=1)
    inp = make_inputs(w)
    with pytest.raises(ValueError):
        OracleRVE(dict(w.desc(), plane_stress=1), inp["grain"], inp["quat"])
    w = small_polycrystal(n=(4, 4, 1), n_grains=2, seed=1)
    inp = make_inputs(w)
    o = OracleRVE(dict(w.desc(), plane_stress=1), inp["grain"], inp["quat"])
    with pytest.raises(ValueError):
        o.step([0, 1e-4, 1e-4, 0, 0, 0], 1.0)
    with pytest.raises(ValueError):
        o.step([0, 1e-4, 0, 0, 0, 0], 1.0, np.zeros(6), 0b000100)
