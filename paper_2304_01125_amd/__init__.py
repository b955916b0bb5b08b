"""MI355X-native solver of one load increment of the FFT crystal-plasticity
phase-field fatigue model (small-strain and finite-strain kinematics), behind the C ABI of
include/rve.h."""
from .rve import (RVE, RvePool, RveError, load, make_desc, FIELDS, FIELD_BITS, RVE_FP64, RVE_MIXED,
                  RVE_MAT_POWER, RVE_MAT_DUNNE, RVE_KIN_SMALL, RVE_KIN_FINITE,
                  RVE_OK, RVE_E_ARG, RVE_E_NOMEM, RVE_E_DEVICE, RVE_E_NOCONV, RVE_E_STATE,
                  rve_footprint_bytes, rve_create, rve_set_microstructure, rve_step_increment,
                  rve_step_increment_mixed, rve_step_increment_finite,
                  rve_fields, rve_destroy, rve_pool_step, exported_symbols)

__all__ = ["RVE", "RvePool", "RveError", "load", "make_desc", "FIELDS", "FIELD_BITS", "RVE_FP64",
           "RVE_MIXED", "RVE_MAT_POWER", "RVE_MAT_DUNNE", "RVE_KIN_SMALL", "RVE_KIN_FINITE", "RVE_OK", "RVE_E_ARG", "RVE_E_NOMEM", "RVE_E_DEVICE", "RVE_E_NOCONV",
           "RVE_E_STATE", "rve_footprint_bytes", "rve_create", "rve_set_microstructure",
           "rve_step_increment", "rve_step_increment_mixed", "rve_step_increment_finite", "rve_fields", "rve_destroy", "rve_pool_step",
           "exported_symbols"]
