"""Host-side checks of the C ABI: every symbol declared in include/rve.h is exported,
argument validation and the footprint are correct.  No GPU call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rve.h")
LIB = os.path.join(ROOT, "paper_2304_01125_amd", "librve.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="librve.so not built")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(rve_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    import paper_2304_01125_amd as p
    lib = p.load()
    names = declared_symbols()
    assert "rve_create" in names and "rve_step_increment" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(p.exported_symbols()) == names


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of rve_desc / rve_stats agree with the C compiler's layout."""
    import shutil
    import subprocess
    from paper_2304_01125_amd.rve import RveDesc, RveStats
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {"rve_desc": RveDesc, "rve_stats": RveStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rve.h"', "int main(void){"]
    for cname, py in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    want = []
    for py in fields.values():
        want.append(ctypes.sizeof(py))
        want.extend(getattr(py, f).offset for f, _ in py._fields_)
    assert got == want


def test_footprint_and_validation():
    import paper_2304_01125_amd as p
    from synth import workload
    w = workload("notched-crystal-16")
    d = p.make_desc(w.desc())
    fp = p.rve_footprint_bytes(d)
    n = 16 ** 3
    assert fp > 65 * n * 8                      # at least the FP64 state
    dm = p.make_desc(w.desc(), p.RVE_MIXED)
    assert p.rve_footprint_bytes(dm) < fp       # FP32 spectral buffers are smaller
    bad = p.make_desc(w.desc())
    bad.n[0] = 10                               # 10 = 2 * 5 is not 2^p 3^q
    assert p.rve_footprint_bytes(bad) == 0
    assert "2^p 3^q" in p.load().rve_last_error().decode()
    bad = p.make_desc(w.desc())
    bad.tol_lin = float("nan")
    assert p.rve_footprint_bytes(bad) == 0


def test_create_rejects_small_or_null_arena():
    import paper_2304_01125_amd as p
    from synth import workload
    lib = p.load()
    d = p.make_desc(workload("notched-crystal-16").desc())
    h = ctypes.c_void_p()
    rc = lib.rve_create(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert rc == p.RVE_E_ARG and not h.value
    fp = p.rve_footprint_bytes(d)
    rc = lib.rve_create(ctypes.byref(d), ctypes.c_void_p(4096), fp - 1, None, ctypes.byref(h))
    assert rc == p.RVE_E_NOMEM


def test_null_handle_calls_fail_cleanly():
    import paper_2304_01125_amd as p
    lib = p.load()
    de = np.zeros(6)
    st = p.rve.RveStats()
    assert lib.rve_step_increment(None, de.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0,
                                  ctypes.byref(st)) == p.RVE_E_ARG
    assert lib.rve_destroy(None) == p.RVE_OK


def test_material_derivative_and_mixed_control_arguments_are_validated():
    import paper_2304_01125_amd as p
    from synth import workload, cmsx4, small_polycrystal
    lib = p.load()
    base = dict(small_polycrystal(n=16, n_grains=4, **cmsx4()).desc(), krylov=1)
    assert p.rve_footprint_bytes(p.make_desc(base)) > 0
    for key, val, msg in [("material", 2, "material"), ("scheme", 3, "deriv"),
                          ("dV", 0.0, "thermally activated"), ("mu", -1.0, "thermally activated"),
                          ("T", float("inf"), "thermally activated"),
                          ("krylov", 2, "krylov"), ("gmres_restart", 0, "gmres_restart"),
                          ("pf_dirichlet", 2, "pf_dirichlet")]:
        d = p.make_desc(dict(base, **{key: val}))
        assert p.rve_footprint_bytes(d) == 0, key
        assert msg in lib.rve_last_error().decode(), (key, lib.rve_last_error())
    big = dict(workload("notched-crystal-16").desc(), n=(1024, 2, 2))
    assert p.rve_footprint_bytes(p.make_desc(big)) == 0
    one = dict(workload("notched-crystal-16").desc(), n=(1, 1, 1))
    assert p.rve_footprint_bytes(p.make_desc(one)) > 0
    de = np.zeros(6)
    dp = de.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = p.rve.RveStats()
    assert lib.rve_step_increment_mixed(None, dp, dp, 61, 1.0, ctypes.byref(st)) == p.RVE_E_ARG


@pytest.mark.parametrize("n", [(16, 16, 16), (128, 128, 128), (256, 256, 256), (512, 512, 16),
                               (512, 384, 128), (384, 512, 256), (512, 512, 512), (2, 2, 2)])
def test_cg_partials_do_not_overlap_the_divergence_partials(n):
    """The CG step writes its block partials while other blocks of the same launch still sum
    the fused divergence pass's (one per block of (N1/2/T) N2 3 blocks, T >= 8, plus one of
    the macro stress): the two ranges of the reduction buffer must be disjoint on every grid
    (512 x 512 x 16 launches 49152 divergence blocks)."""
    import paper_2304_01125_amd as p
    from synth import workload
    lib = p.load()
    for prec in (p.RVE_FP64, p.RVE_MIXED):
        d = p.make_desc(dict(workload("notched-crystal-16").desc(), n=n), prec)
        out = (ctypes.c_int64 * 3)()
        assert lib.rve_diag_partials(ctypes.byref(d), out) == p.RVE_OK
        max_div, cg_off, length = out
        assert max_div >= 3 * (n[0] // 16) * n[1] + 1
        assert cg_off >= max_div
        assert length >= cg_off + 2 * 1024
        # the return map's block partials of the 28 constitutive sums, one per 256 voxels
        assert length >= 28 * ((n[0] * n[1] * n[2] + 255) // 256)
    bad = p.make_desc(dict(workload("notched-crystal-16").desc(), n=(10, 2, 2)))
    assert lib.rve_diag_partials(ctypes.byref(bad), (ctypes.c_int64 * 3)()) == p.RVE_E_ARG


def test_noalloc_rejects_descriptions_beyond_the_static_arena():
    """rve_create_noalloc checks the footprint against its 320 MiB static arena before any
    device call: 128^3 FP64 (about 2 GB) is refused with RVE_E_NOMEM and both sizes."""
    import paper_2304_01125_amd as p
    from synth import workload
    lib = p.load()
    d = p.make_desc(dict(workload("notched-crystal-16").desc(), n=(128, 128, 128)))
    h = ctypes.c_void_p()
    assert lib.rve_create_noalloc(ctypes.byref(d), None, ctypes.byref(h)) == p.RVE_E_NOMEM
    msg = lib.rve_last_error().decode()
    assert "335544320" in msg and str(p.rve_footprint_bytes(d)) in msg
    assert not h.value
    small = p.make_desc(dict(workload("notched-crystal-16").desc(), n=(64, 64, 64)))
    assert p.rve_footprint_bytes(small) <= 335544320
    bad = p.make_desc(dict(workload("notched-crystal-16").desc(), n=(10, 2, 2)))
    assert lib.rve_create_noalloc(ctypes.byref(bad), None, ctypes.byref(h)) == p.RVE_E_ARG


def test_finite_strain_descriptions_are_validated():
    """Finite-strain kinematics run in FP64 with GMRES (the linearised operator is not
    symmetric) and the spectral derivative; anything else is refused on the CPU."""
    import paper_2304_01125_amd as p
    from synth import small_polycrystal
    lib = p.load()
    base = dict(small_polycrystal(n=(8, 6, 4), n_grains=3).desc(), kinematics=1, krylov=1,
                gmres_restart=30)
    fp = p.rve_footprint_bytes(p.make_desc(base))
    small = p.rve_footprint_bytes(p.make_desc(dict(base, kinematics=0)))
    assert fp > small                           # 9-component state and the 81-entry tangent
    for key, val, prec in [("krylov", 0, 0), ("scheme", 1, 0), ("kinematics", 2, 0),
                           ("kinematics", 1, 1)]:
        d = p.make_desc(dict(base, **{key: val}), prec)
        assert p.rve_footprint_bytes(d) == 0, (key, val, prec)
        assert "kinematics" in lib.rve_last_error().decode()
    de = np.zeros(9)
    st = p.rve.RveStats()
    assert lib.rve_step_increment_finite(None, de.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         1.0, ctypes.byref(st)) == p.RVE_E_ARG


def test_gnd_coupling_is_validated():
    import paper_2304_01125_amd as p
    from synth import small_polycrystal, cmsx4
    lib = p.load()
    dunne = small_polycrystal(n=(8, 6, 4), n_grains=3, **cmsx4()).desc()
    assert p.rve_footprint_bytes(p.make_desc(dict(dunne, gnd_coupling=1))) > \
        p.rve_footprint_bytes(p.make_desc(dunne))
    for bad in (dict(dunne, gnd_coupling=2),
                dict(small_polycrystal(n=(8, 6, 4), n_grains=3).desc(), gnd_coupling=1),
                dict(dunne, gnd_coupling=1, kinematics=1, krylov=1)):
        assert p.rve_footprint_bytes(p.make_desc(bad)) == 0
        assert "gnd_coupling" in lib.rve_last_error().decode()


def test_plane_stress_is_validated():
    import paper_2304_01125_amd as p
    from synth import small_polycrystal
    lib = p.load()
    plate = small_polycrystal(n=(8, 6, 1), n_grains=3).desc()
    N = 8 * 6
    assert p.rve_footprint_bytes(p.make_desc(dict(plate, plane_stress=1))) >= \
        p.rve_footprint_bytes(p.make_desc(plate)) + 18 * 8 * N
    for bad in (dict(plate, plane_stress=2),
                dict(small_polycrystal(n=(8, 6, 2), n_grains=3).desc(), plane_stress=1),
                dict(plate, plane_stress=1, kinematics=1, krylov=1)):
        assert p.rve_footprint_bytes(p.make_desc(bad)) == 0
        assert "plane_stress" in lib.rve_last_error().decode()


def test_pool_create_validates_its_arena():
    """rve_pool_create refuses a null arena or one with no 256-byte granule, before any
    device call; pool calls on a null pool are harmless or refused."""
    import paper_2304_01125_amd as p
    lib = p.load()
    h = ctypes.c_void_p()
    assert lib.rve_pool_create(None, 1 << 20, ctypes.byref(h)) == p.RVE_E_ARG
    assert lib.rve_pool_create(ctypes.c_void_p(4096), 100, ctypes.byref(h)) == p.RVE_E_ARG
    assert "granule" in lib.rve_last_error().decode()
    assert lib.rve_pool_destroy(None) == p.RVE_OK
    assert lib.rve_pool_free_bytes(None, None) == 0
    d = p.make_desc(__import__("synth").workload("notched-crystal-16").desc())
    out = ctypes.c_void_p()
    assert lib.rve_create_in_pool(None, ctypes.byref(d), None, ctypes.byref(out)) == p.RVE_E_ARG
    # a pool over an address range the host never dereferences: base rounded up to 256 B,
    # length down to whole granules; a handle larger than the pool, or an invalid
    # description, is refused before any device call, and the empty pool is destroyed
    assert lib.rve_pool_create(ctypes.c_void_p(4096 + 8), 1 << 20, ctypes.byref(h)) == p.RVE_OK
    largest = ctypes.c_size_t(0)
    total = lib.rve_pool_free_bytes(h, ctypes.byref(largest))
    assert total == largest.value == (1 << 20) - 256
    need = p.rve_footprint_bytes(d)
    assert need > total
    assert lib.rve_create_in_pool(h, ctypes.byref(d), None, ctypes.byref(out)) == p.RVE_E_NOMEM
    msg = lib.rve_last_error().decode()
    assert str((need + 255) // 256 * 256) in msg and str(total) in msg, msg
    assert not out.value
    bad = p.make_desc(__import__("synth").workload("notched-crystal-16").desc())
    bad.n[0] = 0
    assert lib.rve_create_in_pool(h, ctypes.byref(bad), None, ctypes.byref(out)) == p.RVE_E_ARG
    assert lib.rve_pool_free_bytes(h, None) == total       # nothing was taken
    assert lib.rve_pool_destroy(h) == p.RVE_OK
