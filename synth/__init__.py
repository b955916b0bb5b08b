"""Seeded synthetic inputs for the periodic-RVE fatigue solver.

This package produces *inputs only*: voxel grain maps, crystal orientations,
per-grain initial strengths, pre-set damage, macroscopic strain histories and
the numeric constants of each workload.  It holds none of the method's
arithmetic (no stiffness, no slip kinematics, no spectral operators), so both
the CPU oracle and the GPU library can take their inputs from here without
sharing any computation.
"""
from .microstructure import (periodic_voronoi, periodic_laguerre, shoemake_quaternions,
                             lognormal_laguerre_weights, notch_mask)
from .loading import triangular_waveform
from .workloads import (Workload, workload, WORKLOADS, make_inputs, small_polycrystal, cmsx4,
                        single_crystal)
from .serving import serving_requests, request_workload

__all__ = ["periodic_voronoi", "periodic_laguerre", "shoemake_quaternions",
           "lognormal_laguerre_weights", "notch_mask", "triangular_waveform", "Workload",
           "workload", "WORKLOADS", "make_inputs", "small_polycrystal", "cmsx4", "single_crystal",
           "serving_requests", "request_workload"]
