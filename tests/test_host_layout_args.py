"""mknn_knn_layout's argument checks come before any GPU work, so they are tested here
without a GPU: a layout other than the two measured ones, and a cloud never uploaded."""
import ctypes

import numpy as np

from paper_2605_02224_amd import _lib


def _call(h, layout):
    return _lib.lib().mknn_knn_layout(h, layout, None, 1, None, None, None)


def test_unknown_layout_is_rejected():
    lib = _lib.lib()
    for layout in (0, 3, -1):
        st = _call(None, layout)
        assert st == -1, st   # MKNN_EINVAL
        assert b"layout" in lib.mknn_last_error()


def test_layout_needs_an_uploaded_cloud():
    lib = _lib.lib()
    pts = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    h = ctypes.c_void_p()
    assert lib.mknn_build(ctypes.c_void_p(pts.ctypes.data), 100, None, ctypes.byref(h)) == 0
    try:
        for layout in (1, 2):
            st = _call(h, layout)
            assert st != 0
            assert b"mknn_knn_layout" in lib.mknn_last_error()
    finally:
        lib.mknn_free(h)
