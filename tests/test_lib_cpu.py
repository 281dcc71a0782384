"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every entry
point declared in include/dysonnet.h, agrees on the parameter count, and rejects invalid
shapes before touching the device."""
import ctypes
import os
import re

import pytest

import dn_inputs as di

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2603_11189_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libdysonnet.so not built")
    return L


def test_header_symbols_are_exported():
    L = _lib()
    hdr = open(os.path.join(ROOT, "include", "dysonnet.h")).read()
    declared = set(re.findall(r"^(?:dn_status|int64_t|const char\*|void)\s+(dn_[a-z_]+)\s*\(", hdr, re.M))
    assert declared == set(L.EXPORTS)
    so = ctypes.CDLL(L.LIB_PATH)
    for name in declared:
        assert hasattr(so, name), name


@pytest.mark.parametrize("name", list(di.WORKLOADS))
def test_param_count_matches_generator(name):
    L = _lib()
    shape = di.WORKLOADS[name].model
    assert L.param_count(shape) == di.param_count(shape)


def test_invalid_shapes_rejected_on_host():
    L = _lib()
    lib = L.lib()
    bad = [
        di.ModelShape(16, 1, 65, 4),      # d > 64
        di.ModelShape(1024, 1, 8, 4),     # N > 512
        di.ModelShape(16, 1, 8, 40),      # s > 32
    ]
    for sh in bad:
        d = L.make_desc(sh, "fp32")
        h = ctypes.c_void_p()
        st = lib.dn_model_create(ctypes.byref(d), ctypes.byref(h))
        assert st == L.DN_EUNSUPPORTED
        assert h.value is None
        assert len(lib.dn_last_error()) > 0
    # d_out != 2
    d = L.make_desc(di.ModelShape(16, 1, 8, 4, d_out=3), "fp32")
    h = ctypes.c_void_p()
    assert lib.dn_model_create(ctypes.byref(d), ctypes.byref(h)) == L.DN_EUNSUPPORTED
    # null descriptor / null handle
    assert lib.dn_model_create(None, ctypes.byref(h)) == L.DN_EINVAL
    d = L.make_desc(di.ModelShape(16, 1, 8, 4), "fp32")
    assert lib.dn_model_create(ctypes.byref(d), None) == L.DN_EINVAL
    # float64 field of one configuration larger than the on-chip tile
    d = L.make_desc(di.ModelShape(512, 1, 64, 4), "fp64")
    assert lib.dn_model_create(ctypes.byref(d), ctypes.byref(h)) == L.DN_EUNSUPPORTED


def test_connected_rejects_bad_arguments_on_host():
    L = _lib()
    lib = L.lib()
    hd = L.make_ham(di.HamSpec("j1j2", "periodic"))
    p = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    # M_max < 2N for J1-J2
    st = lib.dn_connected(ctypes.byref(hd), p, 4, 16, 20, p, p, p, p, None)
    assert st == L.DN_EINVAL and b"M_max" in lib.dn_last_error()
    hd = L.make_ham(di.HamSpec("lrtfim", "open"))
    st = lib.dn_connected(ctypes.byref(hd), p, 4, 16, 8, p, p, p, p, None)
    assert st == L.DN_EINVAL
    st = lib.dn_connected(ctypes.byref(hd), None, 4, 16, 16, p, p, p, p, None)
    assert st == L.DN_EINVAL


def test_bf16_mode_needs_wide_channels_on_host():
    L = _lib()
    lib = L.lib()
    d = L.make_desc(di.ModelShape(32, 2, 16, 8), "bf16")
    h = ctypes.c_void_p()
    assert lib.dn_model_create(ctypes.byref(d), ctypes.byref(h)) == L.DN_EUNSUPPORTED
    assert b"BF16" in lib.dn_last_error()


def test_ragged_and_tuning_entry_points_reject_bad_arguments_on_host():
    L = _lib()
    lib = L.lib()
    # an empty submission is a no-op; a negative count is an error
    assert lib.dn_ragged_eloc(0, None, None, None, None, None, None, 0, 1, None) == L.DN_OK
    assert lib.dn_ragged_eloc(-1, None, None, None, None, None, None, 0, 1, None) == L.DN_EINVAL
    # null arrays, bad stream count and bad mode are caught before any device work
    assert lib.dn_ragged_eloc(1, None, None, None, None, None, None, 0, 1, None) == L.DN_EINVAL
    vp = ctypes.c_void_p
    one = (vp * 1)(16)
    hd = (L.HamDesc * 1)(L.make_ham(di.HamSpec("lrtfim", "open")))
    bb = (ctypes.c_int32 * 1)(4)
    st = lib.dn_ragged_eloc(1, one, hd, one, bb, None, one, 9, 1, None)
    assert st == L.DN_EINVAL and b"n_streams" in lib.dn_last_error()
    st = lib.dn_ragged_eloc(1, one, hd, one, bb, None, one, 0, 7, None)
    assert st == L.DN_EINVAL and b"mode" in lib.dn_last_error()
    h = L.make_ham(di.HamSpec("lrtfim", "open"))
    assert lib.dn_autotune(None, ctypes.byref(h), 16, None, None, None) == L.DN_EINVAL
    assert lib.dn_set_launch_shapes(None, 0, 0) == L.DN_EINVAL
    assert lib.dn_set_product_mode(None, 0) == L.DN_EINVAL
