"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/hsgn.h declares, and argument validation happens on
the host before any device work."""
import ctypes
import os
import re

import pytest

from paper_2606_12162_amd import hsgn as H
from paper_2606_12162_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hsgn.h")).read()
    return sorted(set(re.findall(r"\b(hsgn_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_functions()
    assert decl == sorted(H.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhsgn.so not built")
    L = ctypes.CDLL(H.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_strerror_and_param_validation_on_host():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhsgn.so not built")
    L = H.lib()
    assert L.hsgn_strerror(H.HSGN_ECFL).decode().startswith("Courant")
    bad = H.make_params(W.Params(limiter=7))
    h = ctypes.c_void_p()
    assert L.hsgn_create(ctypes.byref(bad), None, ctypes.byref(h)) == H.HSGN_EINVAL
    for c2 in (-1.0, float("nan")):            # the fixed c^2 must be >= 0
        bad = H.make_params(W.Params(c2=c2))
        assert L.hsgn_create(ctypes.byref(bad), None, ctypes.byref(h)) == H.HSGN_EINVAL
    nosup = H.make_params(W.Params(), precision=5)
    assert L.hsgn_create(ctypes.byref(nosup), None, ctypes.byref(h)) == H.HSGN_ENOTSUP
    good = H.make_params(W.Params())
    assert L.hsgn_create(ctypes.byref(good), None, ctypes.byref(h)) == H.HSGN_OK
    bc = (ctypes.c_int * 4)(0, 1, 1, 1)      # unpaired periodic side
    pid = ctypes.c_int()
    assert L.hsgn_add_grid(h, 0, 0, 16, 16, 0.0, 0.0, 0.1, 0.1, bc, ctypes.byref(pid)) == H.HSGN_EINVAL
    bc = (ctypes.c_int * 4)(1, 1, 1, 1)
    assert L.hsgn_add_grid(h, 0, 0, 3, 16, 0.0, 0.0, 0.1, 0.1, bc, ctypes.byref(pid)) == H.HSGN_EINVAL
    assert L.hsgn_add_grid(h, 0, 0, 16, 16, 0.0, 0.0, 0.1, 0.1, bc, ctypes.byref(pid)) == H.HSGN_OK
    assert L.hsgn_advance(h, 0.0, 1) == H.HSGN_EINVAL          # before finalize
    assert b"finalize" in L.hsgn_last_error(h)
    assert L.hsgn_destroy(h) == H.HSGN_OK


def _patch_set_error(patches):
    """hsgn_finalize of one scenario made of `patches` (level, nx, ny, i0, j0
    in cells of the patch's level, level-0 spacing 1): the status and message.
    Invalid sets are rejected on the host, before any device call."""
    L = H.lib()
    h = ctypes.c_void_p()
    good = H.make_params(W.Params())
    assert L.hsgn_create(ctypes.byref(good), None, ctypes.byref(h)) == H.HSGN_OK
    bc = (ctypes.c_int * 4)(1, 1, 1, 1)
    pid = ctypes.c_int()
    for lev, nx, ny, i0, j0 in patches:
        d = 1.0 / 4 ** lev
        assert L.hsgn_add_grid(h, 0, lev, nx, ny, i0 * d, j0 * d, d, d, bc,
                               ctypes.byref(pid)) == H.HSGN_OK
    rc = L.hsgn_finalize(h)
    msg = L.hsgn_last_error(h).decode()
    L.hsgn_destroy(h)
    return rc, msg


@pytest.mark.parametrize("patches, words", [
    ([(0, 16, 16, 0, 0), (0, 16, 16, 8, 0)], "overlap"),                    # level-0 overlap
    ([(0, 16, 16, 0, 0), (0, 16, 16, 20, 0)], "tile"),                      # hole in level 0
    ([(0, 16, 16, 0, 0), (1, 16, 16, 0, 16)], "domain boundary"),           # touches the edge
    ([(0, 16, 16, 0, 0), (1, 18, 16, 8, 8)], "multiples of 4"),
    ([(0, 16, 16, 0, 0), (1, 16, 16, 10, 8)], "aligned"),                   # not on a coarse corner
    ([(0, 16, 16, 0, 0), (2, 16, 16, 40, 40)], "levels must be dense"),     # no level 1
    ([(0, 32, 32, 0, 0), (1, 16, 16, 20, 20), (2, 16, 16, 80, 80)], "nested"),
])
def test_patch_set_rules_are_checked_on_host(patches, words):
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhsgn.so not built")
    rc, msg = _patch_set_error(patches)
    assert rc == H.HSGN_EINVAL, (rc, msg)
    assert words in msg, msg
