"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function include/fblisa.h declares, and validates geometries on the host."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synthetic as syn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fblisa.h")).read()
    return sorted(set(re.findall(r"FBL_API\s+[\w\s\*]*?\b(fbl?_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fb_lisa_forward", "fb_lisa_backproject", "fb_lisa_step", "fbl_plan_create", "fbl_plan_destroy",
              "fbl_geometry_check", "fbl_last_error"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2605_12085_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTED) == set(_declared())


def test_all_configuration_geometries_are_valid():
    import paper_2605_12085_amd as fbl
    for c in syn.CONFIGS:
        fbl.fbl_geometry_check(syn.config_geometry(c))
    fbl.fbl_geometry_check(syn.tiny_geometry(n=8, det=12, views=16))


@pytest.mark.parametrize("bad,code,needle", [
    (dict(nx=0), 2, "count"),
    (dict(hz=-1.0), 2, "sizes"),
    (dict(du=float("nan")), 2, "sizes"),
    (dict(sdd=400.0), 2, "SDD"),
    (dict(sod=20.0), 2, "between source and detector"),
    (dict(sod=480.0, sdd=500.0), 2, "between source and detector"),
    (dict(nv=64, dv=40.0), 2, "dominant axis is z"),
    (dict(nx=2000, ny=2000, nz=1000), 2, "2^31"),
    (dict(nu=16385, nv=16384, du=0.003, dv=0.003), 2, "2^28"),
])
def test_geometry_rejections(bad, code, needle):
    import paper_2605_12085_amd as fbl
    base = dict(nx=32, ny=32, nz=32, hx=1.0, hy=1.0, hz=1.0, nu=48, nv=48, du=1.0, dv=1.0, sod=500.0, sdd=1000.0,
                n_views=8)
    base.update(bad)
    g = syn.Geometry(**base)
    with pytest.raises(fbl.FblError) as e:
        fbl.fbl_geometry_check(g)
    assert e.value.code == code
    assert needle in str(e.value)


def test_bad_angle_rejected():
    import paper_2605_12085_amd as fbl
    g = syn.Geometry(8, 8, 8, 1.0, 1.0, 1.0, 12, 12, 1.0, 1.0, 500.0, 1000.0, 3, angles=[0.0, float("inf"), 1.0])
    with pytest.raises(fbl.FblError) as e:
        fbl.fbl_geometry_check(g)
    assert "angle" in str(e.value)


def test_null_arguments_fail_before_any_device_work():
    from paper_2605_12085_amd import _lib
    lib = _lib.lib
    assert lib.fbl_geometry_check(None) == _lib.FBL_E_INVALID
    views = (ctypes.c_int32 * 1)(0)
    assert lib.fb_lisa_forward(None, None, views, 1, None, None, None, 1.0, None) == _lib.FBL_E_INVALID
    assert b"plan" in lib.fbl_last_error()
    assert lib.fb_lisa_backproject(None, None, views, 1, 1.0, None, None) == _lib.FBL_E_INVALID
    assert lib.fb_lisa_step(None, None, None, 1.0, 0.0, 0.0, math.inf, None, None, None) == _lib.FBL_E_INVALID
    assert lib.fbl_timing_select(None, 1) == _lib.FBL_E_INVALID
    assert lib.fbl_plan_create(None, 0, 0, 1, None) == _lib.FBL_E_INVALID
    out = ctypes.c_void_p(1)
    assert lib.fbl_plan_create(None, 0, 0, 1, ctypes.byref(out)) == _lib.FBL_E_INVALID
    assert out.value is None
    lib.fbl_plan_destroy(None)


def test_dtype_and_batch_rejections_before_device_work():
    from paper_2605_12085_amd import _lib
    gh = _lib._GeomHolder(syn.tiny_geometry())
    out = ctypes.c_void_p()
    assert _lib.lib.fbl_plan_create(ctypes.byref(gh.s), 7, 0, 4, ctypes.byref(out)) == _lib.FBL_E_DTYPE
    assert _lib.lib.fbl_plan_create(ctypes.byref(gh.s), 0, 3, 4, ctypes.byref(out)) == _lib.FBL_E_DTYPE
    assert _lib.lib.fbl_plan_create(ctypes.byref(gh.s), 0, 0, 0, ctypes.byref(out)) == _lib.FBL_E_RANGE
    assert _lib.lib.fbl_plan_create(ctypes.byref(gh.s), 0, 0, 17, ctypes.byref(out)) == _lib.FBL_E_RANGE


def test_step1_rule_of_the_driver_matches_hand_schedules():
    # the driver's Step 1 is its own code; check it against the same hand-computed
    # sequences that pin the oracle
    import paper_2605_12085_amd as fbl
    path = os.path.join(ROOT, "tests", "golden", "step1_schedules.txt")
    from paper_2605_12085_amd.driver import eps_power
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, seq = line.split(":")
        kind, n, n0, T = head.split()
        n, n0, T = int(n), int(n0), int(T)
        C = fbl.growing_batch_C(n, n0) if kind == "growth" else fbl.constant_batch_C(n, n0, T)
        sizes, k_hat, n_prev = [], 0, n0
        for t in range(T):
            nt = fbl.next_batch_size(n_prev, k_hat, n, n0, n, C, eps_power)
            sizes.append(nt)
            k_hat += math.ceil(n / nt)
            n_prev = nt
        assert sizes == [int(s) for s in seq.split()], line
