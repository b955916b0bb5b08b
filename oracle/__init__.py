"""Plain FP64 CPU oracle of the FFT crystal-plasticity phase-field fatigue increment.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` call it.  It shares no code with the GPU library; its only
common dependency is the seeded input generator package ``synth``.

What it computes (Lucarini, Dunne & Martinez-Paneda, 2023), in the
small-strain specialisation (symmetric strain/stress, 6x6 tangents):

* per-voxel crystal plasticity (Sec. 2.1) with either a power-law flow rule and
  linear hardening, or the thermally activated flow rule (eq. flowrule) with
  Taylor hardening on the SSD and GND densities; backward Euler with the
  strength frozen over the step;
* the hybrid momentum balance div[g(phi) sigma] = 0 solved in Fourier space by
  Newton + GMRES on the displacement correction (Sec. 3.1, eqs. momentum,
  fdef, newton), preconditioned by the inverse acoustic tensor of the
  volume-averaged tangent (eqs. precf, avstiff);
* the AT2 phase-field balance with the stored-energy driving force
  (eqs. strpf, crit, decMiehe, zeta, phase) with the preconditioner of
  eq. precph (read as (1 + l^2 |xi|^2)^-1);
* pointwise plane stress of plates one voxel thick (Sec. 4.1-4.3): the out-of-plane
  stress held at zero at every voxel by a local solve, the in-plane balance on the
  condensed tangent;
* the non-linear alternating minimisation of one time increment (Algorithm 1),
  the history commit (SSD density, plastic work, stored energy density G_s,
  W_crit) and the regularised Nye-tensor GND density (eqs. nye1, the Fourier
  curl, and the regularisation equation of Sec. 3.1).

Every function here uses plain NumPy/SciPy in float64, with no blocking or
fusion beyond the definitions it cites.  Pins against closed forms, brute
force and invariants live in ``tests/test_oracle_*.py``.
"""
from .crystal import (quat_to_rot, cubic_stiffness, rotate4, fcc_slip_systems,
                      screw_directions, to_mandel2, from_mandel2, to_mandel4, from_mandel4,
                      gnd_matrix)
from .constitutive import (GrainTables, return_map, slip_increments, PowerLaw, DunneLaw,
                           flow_law)
from .spectral import Grid
from .mechanics import solve_mechanics, momentum_operator
from .planestress import solve_mechanics_plane, local_plane_stress, condensed_tangent
from .phasefield import split_positive, we_plus, solve_phase_field, solve_phase_field_dirichlet
from .history import nye_tensor, gnd_density
from .increment import OracleRVE

__all__ = ["quat_to_rot", "cubic_stiffness", "rotate4", "fcc_slip_systems", "screw_directions",
           "to_mandel2", "from_mandel2", "to_mandel4", "from_mandel4", "gnd_matrix",
           "GrainTables", "return_map", "slip_increments", "PowerLaw", "DunneLaw", "flow_law", "Grid", "solve_mechanics",
           "momentum_operator", "solve_mechanics_plane", "local_plane_stress", "condensed_tangent",
           "split_positive", "we_plus", "solve_phase_field", "solve_phase_field_dirichlet", "nye_tensor", "gnd_density",
           "OracleRVE"]
