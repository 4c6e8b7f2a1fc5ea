"""The C ABI without a GPU: the library loads, exports every function that
include/librsvd.h declares, and rejects invalid arguments before any device
work, with a message."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "librsvd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:int|void|int64_t|const char\s*\*)\s*(\w+)\s*\(", text, flags=re.M)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["rsvd_truncate", "fullsvd_truncate", "rsvd_plan_create", "rsvd_plan_execute",
              "rsvd_plan_destroy", "rsvd_last_error", "rsvd_plan_profile", "rsvd_gaussian",
              "rsvd_plan_backward", "rsvd_plan_profile_backward", "rsvd_plan_postselect",
              "rsvd_truncate_adaptive", "rsvd_plan_tiles", "rsvd_plan_set_tiles", "rsvd_truncate_noalloc"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1710_01463_amd import _lib
    lib = _lib.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_invalid_arguments_are_rejected_without_a_device():
    from paper_1710_01463_amd import _lib
    lib = _lib.lib()
    vp = ctypes.c_void_p
    dummy = vp(16)  # never dereferenced: validation fails first
    # k = 0
    st = lib.rsvd_truncate(dummy, 0, 10, 10, 10, 0, 2, 1, ctypes.c_uint64(1), 0.0, 0, dummy, 1, dummy,
                           dummy, 10, dummy, dummy, None)
    assert st == _lib.RSVD_ERR_INVALID
    assert b"k" in lib.rsvd_last_error()
    # lda < n
    st = lib.rsvd_truncate(dummy, 0, 10, 10, 5, 2, 2, 1, ctypes.c_uint64(1), 0.0, 0, dummy, 2, dummy,
                           dummy, 10, dummy, dummy, None)
    assert st == _lib.RSVD_ERR_INVALID and b"lda" in lib.rsvd_last_error()
    # negative or NaN delta
    for delta in (-1.0, float("nan")):
        st = lib.rsvd_truncate(dummy, 0, 10, 10, 10, 2, 2, 1, ctypes.c_uint64(1), delta, 0, dummy, 2,
                               dummy, dummy, 10, dummy, dummy, None)
        assert st == _lib.RSVD_ERR_INVALID
    # null input
    st = lib.fullsvd_truncate(None, 0, 10, 10, 10, 2, 0.0, dummy, 2, dummy, dummy, 10, dummy, dummy, None)
    assert st == _lib.RSVD_ERR_INVALID
    # unknown precision / dtype
    st = lib.rsvd_truncate(dummy, 0, 10, 10, 10, 2, 2, 1, ctypes.c_uint64(1), 0.0, 7, dummy, 2, dummy,
                           dummy, 10, dummy, dummy, None)
    assert st == _lib.RSVD_ERR_INVALID
    # plans: empty batch, bad problem
    h = vp()
    assert lib.rsvd_plan_create(None, 0, 0, 0, 0, ctypes.byref(h)) == _lib.RSVD_ERR_INVALID
    probs = (_lib.RsvdProblem * 1)()
    probs[0].m, probs[0].n, probs[0].lda, probs[0].k, probs[0].p, probs[0].q = 8, 8, 8, 3, -1, 1
    assert lib.rsvd_plan_create(probs, 1, 0, 0, 0, ctypes.byref(h)) == _lib.RSVD_ERR_INVALID
    assert b"problem 0" in lib.rsvd_last_error()
    probs[0].p, probs[0].k = 2, 2000
    probs[0].m = probs[0].n = probs[0].lda = 4000
    assert lib.rsvd_plan_create(probs, 1, 0, 0, 0, ctypes.byref(h)) == _lib.RSVD_ERR_INVALID
    lib.rsvd_plan_destroy(None)
    # backward without a plan
    arr = (vp * 1)(16)
    assert lib.rsvd_plan_backward(None, arr, arr, arr, arr, 0.0, None) == _lib.RSVD_ERR_INVALID
    assert b"plan" in lib.rsvd_last_error()
    # adaptive rank: delta must be > 0, k0 <= k_max
    st = lib.rsvd_truncate_adaptive(dummy, 0, 10, 10, 10, 2, 8, 2, 1, ctypes.c_uint64(1), 0.0, 0, dummy, 8,
                                    dummy, dummy, 10, dummy, dummy, None, None)
    assert st == _lib.RSVD_ERR_INVALID and b"delta" in lib.rsvd_last_error()
    st = lib.rsvd_truncate_adaptive(dummy, 0, 10, 10, 10, 9, 8, 2, 1, ctypes.c_uint64(1), 1e-3, 0, dummy, 8,
                                    dummy, dummy, 10, dummy, dummy, None, None)
    assert st == _lib.RSVD_ERR_INVALID
    # post-selection without a plan
    assert lib.rsvd_plan_postselect(None, 4, dummy, None) == _lib.RSVD_ERR_INVALID
    assert b"plan" in lib.rsvd_last_error()
    # allocation-free one-shot: argument checks and the scratch bound come before any device call
    st = lib.rsvd_truncate_noalloc(None, 0, 10, 10, 10, 2, 2, 1, ctypes.c_uint64(1), 0.0, 0, dummy, 2, dummy,
                                   dummy, 10, dummy, dummy, None, None)
    assert st == _lib.RSVD_ERR_INVALID
    st = lib.rsvd_truncate_noalloc(dummy, 0, 10, 10, 10, 0, 2, 1, ctypes.c_uint64(1), 0.0, 0, dummy, 2, dummy,
                                   dummy, 10, dummy, dummy, None, None)
    assert st == _lib.RSVD_ERR_INVALID and b"k" in lib.rsvd_last_error()
    st = lib.rsvd_truncate_noalloc(dummy, 0, 4096, 4096, 4096, 1000, 24, 2, ctypes.c_uint64(1), 0.0, 0, dummy,
                                   1000, dummy, dummy, 4096, dummy, dummy, None, None)
    assert st == _lib.RSVD_ERR_INVALID and b"scratch" in lib.rsvd_last_error()
    # tile query and tile choice without a plan
    count = ctypes.c_int64()
    assert lib.rsvd_plan_tiles(None, None, 0, ctypes.byref(count)) == _lib.RSVD_ERR_INVALID
    assert lib.rsvd_plan_set_tiles(None, None, 0) == _lib.RSVD_ERR_INVALID
    assert b"plan" in lib.rsvd_last_error()


def test_python_layer_fails_loudly_without_the_library(monkeypatch):
    from paper_1710_01463_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librsvd.so"))
    with pytest.raises(ImportError):
        _lib.lib()
