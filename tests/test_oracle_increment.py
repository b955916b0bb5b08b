"""Pins of the oracle's time increment (Algorithm 1) on cases that reduce to a material point."""
import dataclasses
import numpy as np

from oracle import OracleRVE
from oracle.increment import from_tensor6
from synth import single_crystal, make_inputs


def test_homogeneous_crystal_reduces_to_material_point_with_uniform_damage():
    w = dataclasses.replace(single_crystal(n=4, seed=3, notch=False), G_crit=2e-3).parity()
    inp = make_inputs(w)
    r = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    ebar = np.zeros((3, 3))
    triggered_at = None
    for k, (de, dt) in enumerate(zip(inp["deps"][:12], inp["dt"][:12])):
        r.step([0, de, 0, 0, 0, 0], dt)
        ebar[1, 1] += de
        # uniform fields: no fluctuation at all
        assert np.abs(r.eps - ebar[None]).max() <= 1e-15
        for f in (r.phi, r.Gs, r.Wp, r.g):
            assert np.ptp(f) <= 1e-12 * max(1.0, np.abs(f).max())
        if r.trig[0] and triggered_at is None:
            triggered_at = k
    assert triggered_at is not None and triggered_at < 11
    assert r.phi.max() > 0.0


def test_uniform_phase_field_formula_inside_increment():
    # With a homogeneous crystal the driving state S is uniform, and the staggered loop's
    # phase field must equal min(1, max(phi_t, 2S/(1+2S))) with S from the oracle's own
    # energies at the converged strain.
    w = dataclasses.replace(single_crystal(n=4, seed=5, notch=False), G_crit=2e-3).parity()
    inp = make_inputs(w)
    r = OracleRVE(w.desc(), inp["grain"], inp["quat"], inp["tau_c0"], inp["phi0"])
    d = w.desc()
    checked = 0
    for de, dt in zip(inp["deps"][:14], inp["dt"][:14]):
        trig, wcrit, wp, phi_t = r.trig.copy(), r.Wcrit.copy(), r.Wp.copy(), r.phi.copy()
        r.step([0, de, 0, 0, 0, 0], dt)
        if not trig[0]:
            continue
        S = d["ell"] / d["Gc"] * max(0.0, _we_now(r) + r.Wp[0] - wcrit[0])
        expect = min(1.0, max(phi_t[0], 2 * S / (1 + 2 * S)))
        assert abs(r.phi[0] - expect) <= 1e-10
        checked += 1
    assert checked >= 2


def _we_now(r):
    from oracle.phasefield import we_plus
    return we_plus(r.eps[:1] - r.epsp[:1], r.tab.C4[r.gid[:1]])[0]


def test_ratio_rule_zero_over_zero():
    from oracle.increment import _ratio
    assert _ratio(0.0, 0.0) == 0.0
    assert _ratio(1.0, 0.0) == np.inf
    assert _ratio(1.0, 4.0) == 0.25
    assert from_tensor6([1, 2, 3, 4, 5, 6])[0][1, 2] == 4
