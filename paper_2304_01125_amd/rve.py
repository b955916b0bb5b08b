"""Thin ctypes binding of the C ABI declared in include/rve.h.

Only argument marshalling lives here: every step of the increment runs in the HIP
library ``librve.so``.  PyTorch provides the device arena (a uint8 tensor) and
the stream.  The binding refuses to run without the compiled library.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librve.so")

RVE_OK, RVE_E_ARG, RVE_E_NOMEM, RVE_E_DEVICE, RVE_E_NOCONV, RVE_E_STATE = 0, -1, -2, -3, -4, -5
RVE_FP64, RVE_MIXED = 0, 1
RVE_MAT_POWER, RVE_MAT_DUNNE = 0, 1
RVE_KIN_SMALL, RVE_KIN_FINITE = 0, 1

FIELDS = [  # (name, bit, components) in the order rve_fields writes them
    ("strain", 1 << 0, 6), ("stress", 1 << 1, 6), ("stress_eff", 1 << 2, 6),
    ("damage", 1 << 3, 1), ("gs", 1 << 4, 1), ("rho_ssd", 1 << 5, 1), ("rho_gnd", 1 << 6, 1),
    ("wp", 1 << 7, 1), ("h", 1 << 8, 1), ("wcrit", 1 << 9, 1), ("trig", 1 << 10, 1),
    ("eps_p", 1 << 11, 6), ("g", 1 << 12, 1), ("beta_p", 1 << 13, 9),
    # finite-strain handles
    ("defgrad", 1 << 14, 9), ("pk1", 1 << 15, 9), ("fp", 1 << 16, 9),
]
FIELD_BITS = {n: (b, c) for n, b, c in FIELDS}
PASSES = {"fft_z": 0, "fft_y": 1, "x_tangent": 2, "grad": 3, "div": 4, "precond": 5,
          "constitutive": 6, "matvec": 7, "zgrad": 8, "zdiv": 9, "pf_iter": 10}


class RveDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("precision", ctypes.c_int32), ("h", ctypes.c_double),
                ("C11", ctypes.c_double), ("C12", ctypes.c_double), ("C44", ctypes.c_double),
                ("gdot0", ctypes.c_double), ("n_exp", ctypes.c_double),
                ("tau_c0", ctypes.c_double), ("h_lin", ctypes.c_double),
                ("lambda_ssd", ctypes.c_double), ("rho0", ctypes.c_double),
                ("burgers", ctypes.c_double), ("xi_store", ctypes.c_double),
                ("ell", ctypes.c_double), ("Gc", ctypes.c_double), ("G_crit", ctypes.c_double),
                ("k_res", ctypes.c_double), ("ell_fp", ctypes.c_double),
                ("tol_stag", ctypes.c_double), ("tol_newton", ctypes.c_double),
                ("tol_lin", ctypes.c_double), ("max_stag", ctypes.c_int32),
                ("max_newton", ctypes.c_int32), ("max_krylov", ctypes.c_int32),
                ("max_grains", ctypes.c_int32), ("material", ctypes.c_int32),
                ("rho_m", ctypes.c_double), ("v_D", ctypes.c_double), ("dF", ctypes.c_double),
                ("k_B", ctypes.c_double), ("T", ctypes.c_double), ("dV", ctypes.c_double),
                ("mu", ctypes.c_double), ("krylov", ctypes.c_int32),
                ("gmres_restart", ctypes.c_int32), ("deriv", ctypes.c_int32),
                ("pf_dirichlet", ctypes.c_int32), ("kinematics", ctypes.c_int32),
                ("gnd_coupling", ctypes.c_int32), ("plane_stress", ctypes.c_int32)]


class RveStats(ctypes.Structure):
    _fields_ = [("stag_iters", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
                ("krylov_iters", ctypes.c_int32), ("pf_iters", ctypes.c_int32),
                ("ls_cuts", ctypes.c_int32), ("rm_failures", ctypes.c_int32),
                ("macro_stress", ctypes.c_double * 6), ("macro_strain", ctypes.c_double * 6),
                ("max_phi", ctypes.c_double), ("max_phi_slip", ctypes.c_double),
                ("n_triggered", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_constitutive", ctypes.c_double), ("ms_mech_krylov", ctypes.c_double),
                ("ms_phase_field", ctypes.c_double), ("ms_commit", ctypes.c_double),
                ("macro_pk1", ctypes.c_double * 9), ("macro_defgrad", ctypes.c_double * 9),
                ("cg_batch", ctypes.c_double)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def load():
    """Load librve.so (after torch, so that both use the same HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (the HIP runtime must be torch's)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(build it with python paper_2304_01125_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.rve_footprint_bytes.restype = ctypes.c_size_t
    lib.rve_footprint_bytes.argtypes = [ctypes.POINTER(RveDesc)]
    lib.rve_create.restype = ctypes.c_int
    lib.rve_create.argtypes = [ctypes.POINTER(RveDesc), _P, ctypes.c_size_t, _P,
                               ctypes.POINTER(_P)]
    lib.rve_create_noalloc.restype = ctypes.c_int
    lib.rve_create_noalloc.argtypes = [ctypes.POINTER(RveDesc), _P, ctypes.POINTER(_P)]
    lib.rve_set_microstructure.restype = ctypes.c_int
    lib.rve_set_microstructure.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                           _D, _D, _D]
    lib.rve_step_increment.restype = ctypes.c_int
    lib.rve_step_increment.argtypes = [_P, _D, ctypes.c_double, ctypes.POINTER(RveStats)]
    lib.rve_diag_time_pass.restype = ctypes.c_int
    lib.rve_diag_time_pass.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
    lib.rve_diag_pass_time.restype = ctypes.c_int
    lib.rve_diag_pass_time.argtypes = [_P, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.rve_step_increment_mixed.restype = ctypes.c_int
    lib.rve_step_increment_mixed.argtypes = [_P, _D, _D, ctypes.c_int32, ctypes.c_double,
                                             ctypes.POINTER(RveStats)]
    lib.rve_fields.restype = ctypes.c_int
    lib.rve_fields.argtypes = [_P, ctypes.c_uint32, _D, ctypes.c_size_t]
    lib.rve_fields_count.restype = ctypes.c_size_t
    lib.rve_fields_count.argtypes = [_P, ctypes.c_uint32]
    lib.rve_destroy.restype = ctypes.c_int
    lib.rve_destroy.argtypes = [_P]
    lib.rve_last_error.restype = ctypes.c_char_p
    lib.rve_last_error.argtypes = []
    for name in ("rve_diag_rfft", "rve_diag_irfft"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [_P, ctypes.c_int32, _D, _D]
    lib.rve_diag_constitutive.restype = ctypes.c_int
    lib.rve_diag_constitutive.argtypes = [_P, _D, ctypes.c_double, _D, _D]
    lib.rve_diag_pass.restype = ctypes.c_int
    lib.rve_diag_pass.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, _D]
    lib.rve_pool_step.restype = ctypes.c_int
    lib.rve_pool_step.argtypes = [ctypes.POINTER(_P), ctypes.c_int32, _D, _D,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(RveStats)]
    lib.rve_pool_create.restype = ctypes.c_int
    lib.rve_pool_create.argtypes = [_P, ctypes.c_size_t, ctypes.POINTER(_P)]
    lib.rve_create_in_pool.restype = ctypes.c_int
    lib.rve_create_in_pool.argtypes = [_P, ctypes.POINTER(RveDesc), _P, ctypes.POINTER(_P)]
    lib.rve_pool_free_bytes.restype = ctypes.c_size_t
    lib.rve_pool_free_bytes.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
    lib.rve_pool_destroy.restype = ctypes.c_int
    lib.rve_pool_destroy.argtypes = [_P]
    lib.rve_diag_partials.restype = ctypes.c_int
    lib.rve_diag_partials.argtypes = [ctypes.POINTER(RveDesc), ctypes.POINTER(ctypes.c_int64)]
    lib.rve_step_increment_finite.restype = ctypes.c_int
    lib.rve_step_increment_finite.argtypes = [_P, _D, ctypes.c_double, ctypes.POINTER(RveStats)]
    lib.rve_diag_constitutive_finite.restype = ctypes.c_int
    lib.rve_diag_constitutive_finite.argtypes = [_P, _D, ctypes.c_double, _D, _D]
    lib.rve_diag_operator.restype = ctypes.c_int
    lib.rve_diag_operator.argtypes = [_P, _D, _D]
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C ABI entry points (as declared in include/rve.h)."""
    return ["rve_footprint_bytes", "rve_create", "rve_create_noalloc", "rve_set_microstructure", "rve_step_increment",
            "rve_step_increment_mixed", "rve_step_increment_finite", "rve_fields", "rve_fields_count", "rve_destroy", "rve_last_error", "rve_diag_rfft",
            "rve_diag_irfft", "rve_diag_constitutive", "rve_diag_constitutive_finite",
            "rve_diag_operator", "rve_diag_pass",
            "rve_diag_time_pass", "rve_diag_pass_time", "rve_diag_partials",
            "rve_pool_step", "rve_pool_create", "rve_create_in_pool", "rve_pool_free_bytes",
            "rve_pool_destroy"]


class RveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rve error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != RVE_OK:
        raise RveError(rc, load().rve_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def make_desc(desc, precision=RVE_FP64, max_grains=4096):
    d = RveDesc()
    for a in range(3):
        d.n[a] = int(desc["n"][a])
    d.precision = int(precision)
    for k in ("h", "C11", "C12", "C44", "gdot0", "n_exp", "tau_c0", "h_lin", "lambda_ssd", "rho0",
              "burgers", "xi_store", "ell", "Gc", "G_crit", "k_res", "ell_fp", "tol_stag",
              "tol_newton", "tol_lin"):
        setattr(d, k, float(desc[k]))
    d.max_stag = int(desc["max_stag"])
    d.max_newton = int(desc["max_newton"])
    d.max_krylov = int(desc["max_krylov"])
    d.max_grains = int(max_grains)
    d.deriv = int(desc.get("scheme", 0))
    d.pf_dirichlet = int(desc.get("pf_dirichlet", 0))
    d.krylov = int(desc.get("krylov", 0))
    d.gmres_restart = int(desc.get("gmres_restart", 30))
    d.material = int(desc.get("material", RVE_MAT_POWER))
    d.kinematics = int(desc.get("kinematics", RVE_KIN_SMALL))
    d.gnd_coupling = int(desc.get("gnd_coupling", 0))
    d.plane_stress = int(desc.get("plane_stress", 0))
    if d.material == RVE_MAT_DUNNE:
        for k in ("rho_m", "v_D", "dF", "k_B", "T", "dV", "mu"):
            setattr(d, k, float(desc[k]))
    return d


def rve_footprint_bytes(d):
    return load().rve_footprint_bytes(ctypes.byref(d))


def rve_create(d, arena_ptr, arena_bytes, stream_ptr):
    h = _P()
    _check(load().rve_create(ctypes.byref(d), _P(arena_ptr), arena_bytes, _P(stream_ptr),
                             ctypes.byref(h)))
    return h


def rve_set_microstructure(h, grain, quat, tau_c0=None, phi0=None):
    g = np.ascontiguousarray(grain, dtype=np.int32)
    q = np.ascontiguousarray(quat, dtype=np.float64).reshape(-1, 4)
    t = None if tau_c0 is None else np.ascontiguousarray(tau_c0, dtype=np.float64)
    p = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64)
    _check(load().rve_set_microstructure(h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         len(q), _dptr(q), _dptr(t), _dptr(p)))


def rve_step_increment(h, deps6, dt):
    de = np.ascontiguousarray(deps6, dtype=np.float64)
    st = RveStats()
    rc = load().rve_step_increment(h, _dptr(de), float(dt), ctypes.byref(st))
    return rc, st.as_dict()


def rve_step_increment_mixed(h, deps6, dsig6, stress_mask, dt):
    de = np.ascontiguousarray(deps6, dtype=np.float64)
    ds = np.ascontiguousarray(np.zeros(6) if dsig6 is None else dsig6, dtype=np.float64)
    st = RveStats()
    rc = load().rve_step_increment_mixed(h, _dptr(de), _dptr(ds), int(stress_mask), float(dt),
                                         ctypes.byref(st))
    return rc, st.as_dict()


def rve_step_increment_finite(h, dF9, dt):
    d = np.ascontiguousarray(np.asarray(dF9, dtype=np.float64).reshape(9))
    st = RveStats()
    rc = load().rve_step_increment_finite(h, _dptr(d), float(dt), ctypes.byref(st))
    return rc, st.as_dict()


def rve_fields(h, mask, nvox):
    n = load().rve_fields_count(h, mask)
    out = np.empty(n, dtype=np.float64)
    _check(load().rve_fields(h, mask, _dptr(out), n))
    return out


def rve_destroy(h):
    return load().rve_destroy(h)


def rve_pool_step(handles, deps, dt):
    """One concurrent increment of several handles; returns (rc, status list, stats list)."""
    n = len(handles)
    arr = (_P * n)(*[h.value if isinstance(h, _P) else h for h in handles])
    de = np.ascontiguousarray(np.asarray(deps, dtype=np.float64).reshape(n, 6))
    d = np.ascontiguousarray(np.asarray(dt, dtype=np.float64).reshape(n))
    status = (ctypes.c_int32 * n)()
    stats = (RveStats * n)()
    rc = load().rve_pool_step(arr, n, _dptr(de), _dptr(d), status, stats)
    return rc, list(status), [s.as_dict() for s in stats]


class RvePool:
    """A serving pool (rve_pool_create): one torch-allocated device arena of budget_bytes
    from which RVE(..., pool=...) handles take their footprint and to which they return it
    at close()."""

    def __init__(self, budget_bytes, device=0):
        import torch
        lib = load()
        self.device = torch.device("cuda", device)
        self.arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.h = _P()
        _check(lib.rve_pool_create(_P(self.arena.data_ptr()), int(budget_bytes),
                                   ctypes.byref(self.h)))

    def free_bytes(self):
        """(total free bytes, largest free range)"""
        largest = ctypes.c_size_t(0)
        tot = load().rve_pool_free_bytes(self.h, ctypes.byref(largest))
        return int(tot), int(largest.value)

    def close(self):
        if getattr(self, "h", None):
            _check(load().rve_pool_destroy(self.h))
            self.h = None


class RVE:
    """One periodic RVE solved on the GPU.  ``desc`` is the flat dict of
    ``synth.Workload.desc()``; precision is RVE_FP64 or RVE_MIXED."""

    def __init__(self, desc, precision=RVE_FP64, device=0, stream=None, max_grains=4096,
                 noalloc=False, pool=None):
        """noalloc: create the handle with rve_create_noalloc (the library's static device
        arena, one such handle per device at a time) instead of a torch-allocated arena;
        pool: an RvePool whose arena holds the handle (rve_create_in_pool)."""
        import torch
        lib = load()
        self.desc = dict(desc)
        self.n = tuple(int(v) for v in desc["n"])
        self.nvox = int(np.prod(self.n))
        self._d = make_desc(desc, precision, max_grains)
        nbytes = lib.rve_footprint_bytes(ctypes.byref(self._d))
        if nbytes == 0:
            raise RveError(RVE_E_ARG, lib.rve_last_error().decode())
        self.device = torch.device("cuda", device)
        if noalloc:
            torch.cuda.set_device(self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.arena = None
            h = _P()
            _check(lib.rve_create_noalloc(ctypes.byref(self._d), _P(self.stream.cuda_stream),
                                          ctypes.byref(h)))
            self.h = h
            self.footprint = nbytes
            return
        if pool is not None:
            torch.cuda.set_device(self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.arena = None
            self.pool = pool            # the pool's arena outlives the handle
            h = _P()
            _check(lib.rve_create_in_pool(pool.h, ctypes.byref(self._d),
                                          _P(self.stream.cuda_stream), ctypes.byref(h)))
            self.h = h
            self.footprint = nbytes
            return
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        # the library works on its own stream (default priority), so that its CG
        # iterations can be replayed as HIP graphs; that stream first waits for the
        # work torch has queued on the arena's allocation stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.h = rve_create(self._d, self.arena.data_ptr(), nbytes, self.stream.cuda_stream)
        self.footprint = nbytes

    def set_microstructure(self, grain, quat, tau_c0=None, phi0=None):
        rve_set_microstructure(self.h, grain, quat, tau_c0, phi0)

    def step(self, deps6, dt, check=True, dsig6=None, stress_mask=0):
        """One increment; components with bit c of stress_mask set follow the macro stress
        increment dsig6[c] (mixed control), the others the strain increment deps6[c]."""
        if stress_mask:
            rc, st = rve_step_increment_mixed(self.h, deps6, dsig6, stress_mask, dt)
        else:
            rc, st = rve_step_increment(self.h, deps6, dt)
        st["status"] = rc
        if check:
            _check(rc)
        return st

    def step_finite(self, dF9, dt, check=True):
        """One finite-strain increment under the macro deformation gradient increment dF9
        (3x3 row-major)."""
        rc, st = rve_step_increment_finite(self.h, dF9, dt)
        st["status"] = rc
        if check:
            _check(rc)
        return st

    def fields(self, names=("strain", "stress", "damage")):
        mask = 0
        for nm in names:
            mask |= FIELD_BITS[nm][0]
        flat = rve_fields(self.h, mask, self.nvox)
        out, off = {}, 0
        for nm, bit, nc in FIELDS:
            if mask & bit:
                blk = flat[off:off + nc * self.nvox]
                out[nm] = blk.reshape(nc, self.nvox).T.copy() if nc > 1 else blk.copy()
                off += nc * self.nvox
        return out

    # diagnostics ---------------------------------------------------------------------
    def rfft(self, real, ncomp):
        nh = (self.n[0] // 2 + 1) * self.n[1] * self.n[2]
        a = np.ascontiguousarray(real, dtype=np.float64).ravel()
        out = np.empty(2 * nh * ncomp)
        _check(load().rve_diag_rfft(self.h, ncomp, _dptr(a), _dptr(out)))
        return out.view(np.complex128).reshape(ncomp, nh)

    def irfft(self, spec, ncomp):
        s = np.ascontiguousarray(spec, dtype=np.complex128).ravel().view(np.float64)
        out = np.empty(ncomp * self.nvox)
        _check(load().rve_diag_irfft(self.h, ncomp, _dptr(s), _dptr(out)))
        return out.reshape(ncomp, self.nvox)

    def constitutive(self, eps6, dt):
        e = np.ascontiguousarray(np.asarray(eps6, dtype=np.float64).T).ravel()
        sig = np.empty(6 * self.nvox)
        gk = np.empty(21 * self.nvox)
        _check(load().rve_diag_constitutive(self.h, _dptr(e), float(dt), _dptr(sig), _dptr(gk)))
        return sig.reshape(6, self.nvox).T, gk.reshape(21, self.nvox).T

    def constitutive_finite(self, F9, dt):
        """Finite-strain return map at deformation gradients F9 (M x 9, row-major): the
        effective first Piola-Kirchhoff stress (M x 9) and g(phi) dP/dF (M x 9 x 9)."""
        f = np.ascontiguousarray(np.asarray(F9, dtype=np.float64).reshape(self.nvox, 9).T).ravel()
        P = np.empty(9 * self.nvox)
        K = np.empty(81 * self.nvox)
        _check(load().rve_diag_constitutive_finite(self.h, _dptr(f), float(dt), _dptr(P), _dptr(K)))
        return P.reshape(9, self.nvox).T, K.reshape(9, 9, self.nvox).transpose(2, 0, 1)

    def time_pass(self, name="x_tangent", on=True, every=1):
        """Live timing of a kernel inside the solver's CG iterations (HIP events on the
        handle's stream) in every `every`-th iteration of each solve; the timed
        iterations are launched eagerly."""
        _check(load().rve_diag_time_pass(self.h, PASSES[name], int(every) if on else 0))

    def pass_time(self):
        """(timed launches, their summed ms) since the previous call."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(load().rve_diag_pass_time(self.h, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def operator(self, u3):
        u = np.ascontiguousarray(np.asarray(u3, dtype=np.float64).T).ravel()
        v = np.empty(3 * self.nvox)
        _check(load().rve_diag_operator(self.h, _dptr(u), _dptr(v)))
        return v.reshape(3, self.nvox).T

    def launch_pass(self, pass_id, reps):
        """Enqueue `reps` launches of one operator building block on the handle's stream
        (no synchronisation); returns the algorithmic bytes of one launch."""
        b = ctypes.c_double(0.0)
        _check(load().rve_diag_pass(self.h, int(pass_id), int(reps), ctypes.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "h", None):
            rve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
