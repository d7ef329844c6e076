"""The C-ABI library loads, exports what include/ckv.h declares, and rejects bad
arguments on the host (no GPU work is started by any call here)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2006_14927_amd import ckv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ckv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckv_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ckv.LIB_PATH):
        pytest.fail("libckv.so not built (run __graft_entry__.build())")
    return ckv.lib()


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(ckv.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_version(L):
    assert L.ckv_version() == 114


def test_struct_sizes_match_header_layout():
    assert C.sizeof(ckv._Segments) == 12 * 8
    assert C.sizeof(ckv._Params) == 4 * 8 + 8 + 4 * 4 + 2 * 8 + 8 + 2 * 4 + 8
    assert C.sizeof(ckv._Result) == 5 * 8 + 8 * 8 + 8 + 4 * 4
    assert C.sizeof(ckv._Cursor) == 16
    assert C.sizeof(ckv._Output) == 7 * 8
    assert C.sizeof(ckv._SoftList) == 3 * 8


def _atmo_create(L, alt, eta, obs=2200.0, step=0.0):
    alt = np.ascontiguousarray(alt, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    h = C.c_void_p()
    rc = L.ckv_atmo_create(ckv._np_ptr(alt), ckv._np_ptr(eta), alt.shape[0], obs, step, C.byref(h))
    return rc, h


@pytest.mark.parametrize("alt,eta,obs,step,code", [
    ([0.0], [1e-4], 0.0, 0.0, -1),                                  # too few points
    ([0.0, 100.0, 100.0], [3e-4, 2e-4, 1e-4], 0.0, 0.0, -2),        # not increasing
    ([0.0, 100.0, 200.0], [3e-4, -2e-4, 1e-4], 0.0, 0.0, -2),       # eta < 0
    ([0.0, 100.0, 200.0], [3e-4, np.nan, 1e-4], 0.0, 0.0, -2),      # non-finite
    ([0.0, 100.0, 200.0], [3e-4, 2e-4, 1e-4], 500.0, 0.0, -2),      # obs above table
    ([0.0, 100.0, 200.0], [3e-4, 2e-4, 1e-4], 0.0, -1.0, -1),       # negative step
    ([0.0, 100.0, 200.0], [3e-4, 2e-4, 1e-4], 150.0, 100.0, -2),    # one node only
])
def test_atmosphere_validation(L, alt, eta, obs, step, code):
    rc, h = _atmo_create(L, alt, eta, obs, step)
    assert rc == code
    assert not h.value
    assert L.ckv_last_error()


def test_depth_table_validation(L):
    alt = np.array([0.0, 100.0, 200.0])
    eta = np.array([3e-4, 2e-4, 1e-4])
    h = C.c_void_p()
    for depth in (np.array([1000.0, 1001.0, 900.0]), np.array([1000.0, np.inf, 900.0])):
        rc = L.ckv_atmo_create_with_depth(ckv._np_ptr(alt), ckv._np_ptr(eta), ckv._np_ptr(depth), 3,
                                          0.0, 0.0, C.byref(h))
        assert rc == -2 and not h.value and L.ckv_last_error()
    nb = C.c_int32()
    assert L.ckv_profile_bins(None, 10.0, C.byref(nb)) == -1
    assert L.ckv_atmo_depth(None, None) == -1
    with pytest.raises(ckv.CkvError):
        ckv.Streamer(None, None, None, ckv.make_params(depth_bin=10.0))


def test_array_validation(L):
    h = C.c_void_p()
    x = np.zeros(2)
    r = np.array([1.0, 0.0])
    assert L.ckv_array_create(ckv._np_ptr(x), ckv._np_ptr(x), ckv._np_ptr(r), 2, C.byref(h)) == -2
    assert L.ckv_array_create(ckv._np_ptr(x), ckv._np_ptr(x), ckv._np_ptr(r), 0, C.byref(h)) == -1
    assert L.ckv_array_create(None, ckv._np_ptr(x), ckv._np_ptr(r), 2, C.byref(h)) == -1


def test_workspace_size_grows_with_inputs(L):
    p = ckv.make_params()
    a = ckv.workspace_size(1000, 1, 9, 1000, p)
    b = ckv.workspace_size(100000, 1, 9, 1000, p)
    c = ckv.workspace_size(100000, 1, 9, 10**6, p)
    assert 0 < a < b < c
    assert L.ckv_workspace_size(-1, 1, 9, 0, C.byref(p)) == 0


def test_run_argument_validation(L):
    segs = ckv._Segments(*([None] * 10), 5, None)       # n > 0 with NULL arrays
    sh = ckv._Showers(None, None, None, None, 1)
    out = ckv._Output(None, None, 0, None, None)
    p = ckv.make_params()
    rc = L.ckv_run(C.byref(segs), C.byref(sh), C.byref(p), None, None, None, 0, C.byref(out), None,
                   None)
    assert rc == -1
    bad_reserved = ckv.make_params()
    bad_reserved.reserved = 1
    for bad in (ckv.make_params(bunch_size=0.0), ckv.make_params(lambda_min=600.0),
                ckv.make_params(precision=7), ckv.make_params(w_min=1.5),
                ckv.make_params(tile_segments=65), ckv.make_params(depth_bin=-1.0), bad_reserved,
                ckv.make_params(earth_radius=-1.0), ckv.make_params(earth_radius=float("inf")),
                ckv.make_params(earth_radius=6.371e6, tile_segments=16),
                ckv.make_params(earth_radius=6.371e6, depth_bin=10.0),
                ckv.make_params(earth_radius=6.371e6, grazing_exact=True)):
        empty = ckv._Segments(*([None] * 10), 0, None)
        assert L.ckv_run(C.byref(empty), C.byref(sh), C.byref(bad), None, None, None, 0,
                         C.byref(out), None, None) == -1
