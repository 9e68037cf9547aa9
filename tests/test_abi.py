"""The C interface: the library loads and exports every declared entry point,
and host-side argument checks reject bad calls before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tpcx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tpcx_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2601_20569_amd as px
    from paper_2601_20569_amd import build as B
    if B.is_stale():
        B.build()
    return px.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 7, names
    for n in names:
        assert hasattr(lib, n), n


def test_host_argument_checks(lib):
    import paper_2601_20569_amd as px
    h = ctypes.c_void_p()
    assert lib.tpcx_create(None, None, None, ctypes.byref(h)) == px.TPCX_E_ARG
    xs = (ctypes.c_float * 3)(100.0, 99.0, 101.0)  # not increasing
    g = px.Geometry(3, ctypes.cast(xs, ctypes.POINTER(ctypes.c_float)), 0.17, 0.5)
    p = px.MethodParams().c_struct()
    assert lib.tpcx_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == px.TPCX_E_ARG
    xs = (ctypes.c_float * 3)(100.0, 101.0, 102.0)
    g = px.Geometry(3, ctypes.cast(xs, ctypes.POINTER(ctypes.c_float)), 0.17, 0.5)
    bad = px.MethodParams(sinphi_max=1.5).c_struct()
    assert lib.tpcx_create(ctypes.byref(g), ctypes.byref(bad), None, ctypes.byref(h)) == px.TPCX_E_ARG
    t = px.Tuning(2.0, 0, 256, 16, 16, 0, 16)  # zero z bins
    assert lib.tpcx_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(t), ctypes.byref(h)) == px.TPCX_E_ARG
    t = px.Tuning(2.0, 8, 256, 16, 65, 0, 16)  # refill threshold above the wavefront width
    assert lib.tpcx_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(t), ctypes.byref(h)) == px.TPCX_E_ARG
    t = px.Tuning(2.0, 8, 256, 16, 16, -1, 16)  # negative refit grid
    assert lib.tpcx_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(t), ctypes.byref(h)) == px.TPCX_E_ARG
    assert lib.tpcx_workspace_bytes(None, 1, 10, 1) == 0
    assert lib.tpcx_batched_workspace_bytes(None, 1, 10, 1, 1, 1) == 0
    assert lib.tpcx_autotune_workspace_bytes(None, 1, 10, 1, 1, 1) == 0
    assert lib.tpcx_refit_workspace_bytes(None, 1, 1) == 0
    assert lib.tpcx_set_tuning(None, None) == px.TPCX_E_ARG
    assert lib.tpcx_track_batched(None, None, None, 0, 0, None, None, None) == px.TPCX_E_ARG
    assert lib.tpcx_autotune_batched(None, None, None, 0, 0, None, None, 1, None, None) == px.TPCX_E_ARG
    assert lib.tpcx_refit(None, None, None, None, None, None, 0, None) == px.TPCX_E_ARG
    assert lib.tpcx_refit_backward(None, None, None, None, None, 0, None) == px.TPCX_E_ARG
    assert lib.tpcx_timing_enable(None, 1) == px.TPCX_E_ARG
    assert lib.tpcx_track(None, None, None, 0, 0, None, None, None) == px.TPCX_E_ARG
    assert lib.tpcx_poll(None, None, None) == px.TPCX_E_ARG
    assert lib.tpcx_strerror(px.TPCX_E_CAPACITY).startswith(b"a device capacity")


def test_default_tuning_is_valid(lib):
    import paper_2601_20569_amd as px
    for u, n in ((1, 0), (1, 20000), (36, 2_000_000), (576, 700_000_000)):
        t = px.default_tuning(u, n)
        assert 1 <= t.n_zbins <= 65536 and t.block % 64 == 0 and t.bin_y > 0
        assert 1 <= t.construct_refill <= 64 and 1 <= t.refit_refill <= 64 and t.refit_grid >= 0
