"""mknn_build_device's argument checks and small-cloud path run before any GPU work, so
they are tested here without a GPU: errors as mknn_build's, the 2^21 - 2 site limit of the
ridge keys, and clouds of fewer than five points handed to the host construction (same
lists)."""
import ctypes

import numpy as np
import pytest

from paper_2605_02224_amd import _lib


def _build_device(pts, order=None):
    lib = _lib.lib()
    h = ctypes.c_void_p()
    p = None if pts is None else ctypes.c_void_p(pts.ctypes.data)
    o = None if order is None else ctypes.c_void_p(order.ctypes.data)
    n = 0 if pts is None else pts.shape[0]
    st = lib.mknn_build_device(p, n, o, None, ctypes.byref(h))
    return st, h


def _lists(h):
    lib = _lib.lib()
    off = ctypes.c_void_p()
    ent = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    assert lib.mknn_successors(h, ctypes.byref(off), ctypes.byref(ent), ctypes.byref(nnz)) == 0
    n = lib.mknn_size(h)
    o = np.ctypeslib.as_array(ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
    e = (np.ctypeslib.as_array(ctypes.cast(ent, ctypes.POINTER(ctypes.c_int32)), (nnz.value,)).copy()
         if nnz.value else np.zeros(0, np.int32))
    return o, e


def test_rejects_bad_arguments():
    pts = np.random.default_rng(0).standard_normal((100, 3)).astype(np.float32)
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.mknn_build_device(ctypes.c_void_p(pts.ctypes.data), 0, None, None,
                                 ctypes.byref(h)) == _lib.EINVAL
    assert lib.mknn_build_device(None, 10, None, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.mknn_build_device(ctypes.c_void_p(pts.ctypes.data), 100, None, None,
                                 None) == _lib.EINVAL
    bad = np.arange(100, dtype=np.int32)
    bad[5] = 7
    assert _build_device(pts, bad)[0] == _lib.EINVAL
    nan = pts.copy()
    nan[17, 1] = np.nan
    st, _ = _build_device(nan)
    assert st == _lib.ENONFINITE
    assert "point 17" in lib.mknn_last_error().decode()


def test_site_limit_of_the_ridge_keys():
    n = (1 << 21) - 1
    pts = np.zeros((n, 3), np.float32)   # never read: the size check comes first
    st, _ = _build_device(pts)
    assert st == _lib.EUNSUPPORTED
    assert "2^21" in _lib.lib().mknn_last_error().decode()


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_small_clouds_take_the_host_construction(n):
    pts = np.random.default_rng(n).standard_normal((n, 3)).astype(np.float32)
    st, h = _build_device(pts)
    assert st == _lib.OK
    ref = ctypes.c_void_p()
    assert _lib.lib().mknn_build(ctypes.c_void_p(pts.ctypes.data), n, None,
                                 ctypes.byref(ref)) == _lib.OK
    a, b = _lists(h), _lists(ref)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = (ctypes.c_int64 * 6)()
    assert _lib.lib().mknn_build_device_stats(c, None) == _lib.OK
    assert list(c) == [0] * 6   # the device path did not run
    _lib.lib().mknn_free(h)
    _lib.lib().mknn_free(ref)
