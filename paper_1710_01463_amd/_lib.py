"""ctypes loader for librsvd.so (argument marshalling only).

The library must have been built for gfx950 (python -m paper_1710_01463_amd.build);
there is no fallback: a missing library is an error.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsvd.so")

RSVD_OK, RSVD_ERR_INVALID, RSVD_ERR_ALLOC, RSVD_ERR_HIP, RSVD_ERR_NONFINITE, RSVD_ERR_NOCONV = 0, -1, -2, -3, -4, -5
RSVD_ERR_SINGULAR = -6
RSVD_F64, RSVD_F32 = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2}
PLAN_FULLSVD, PLAN_GRAPH, PLAN_SAVE, PLAN_NO_REFINE, PLAN_TUNE, PLAN_ROUND_LAUNCHES = 1, 2, 4, 8, 16, 32
PLAN_BLOCK_KRYLOV, PLAN_COMPLEX, PLAN_BLOCKED_QR, PLAN_SINGLE_VIEW, PLAN_FP64_FINAL = 64, 128, 256, 512, 1024

PHASES = ["stage", "omega", "sketch", "gram", "chol", "trsm", "householder", "project", "jacobi",
          "finish", "backproj", "signfix", "other", "bw_gemm", "bw_small"]

STATUS_NAMES = {0: "ok", -1: "invalid argument", -2: "allocation failed", -3: "HIP error",
                -4: "non-finite input", -5: "Jacobi did not converge"}


class RsvdProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("k", ctypes.c_int64), ("p", ctypes.c_int64), ("q", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("delta_trunc", ctypes.c_double),
                ("ldu", ctypes.c_int64), ("ldvt", ctypes.c_int64)]


class RsvdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librsvd: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1710_01463_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        L.rsvd_truncate.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _i64,
                                    ctypes.c_uint64, ctypes.c_double, ctypes.c_int, _vp, _i64, _vp,
                                    _vp, _i64, _vp, _vp, _vp]
        L.rsvd_truncate.restype = ctypes.c_int
        L.rsvd_truncate_noalloc.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _i64,
                                            ctypes.c_uint64, ctypes.c_double, ctypes.c_int, _vp, _i64, _vp,
                                            _vp, _i64, _vp, _vp, _vp, _vp]
        L.rsvd_truncate_noalloc.restype = ctypes.c_int
        L.rsvd_truncate_adaptive.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, _i64, _i64, _i64,
                                             ctypes.c_uint64, ctypes.c_double, ctypes.c_int, _vp, _i64, _vp,
                                             _vp, _i64, _vp, _vp, ctypes.POINTER(ctypes.c_int), _vp]
        L.rsvd_truncate_adaptive.restype = ctypes.c_int
        L.fullsvd_truncate.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _i64, ctypes.c_double,
                                       _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp]
        L.fullsvd_truncate.restype = ctypes.c_int
        L.rsvd_gaussian.argtypes = [ctypes.c_uint64, _i64, _i64, _vp, _vp]
        L.rsvd_gaussian.restype = ctypes.c_int
        L.rsvd_philox4x32_10.argtypes = [_vp, _vp, _i64, _vp]
        L.rsvd_philox4x32_10.restype = ctypes.c_int
        L.rsvd_plan_create.argtypes = [ctypes.POINTER(RsvdProblem), _i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint, ctypes.POINTER(_vp)]
        L.rsvd_plan_create.restype = ctypes.c_int
        L.rsvd_plan_execute.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp, _vp, _vp]
        L.rsvd_plan_execute.restype = ctypes.c_int
        L.rsvd_plan_profile.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp, _vp,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int, _vp]
        L.rsvd_plan_profile.restype = ctypes.c_int
        _pp = ctypes.POINTER(_vp)
        L.rsvd_plan_backward.argtypes = [_vp, _pp, _pp, _pp, _pp, ctypes.c_double, _vp]
        L.rsvd_plan_backward.restype = ctypes.c_int
        L.rsvd_plan_profile_backward.argtypes = [_vp, _pp, _pp, _pp, _pp, ctypes.c_double,
                                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64),
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int, _vp]
        L.rsvd_plan_profile_backward.restype = ctypes.c_int
        L.rsvd_plan_postselect.argtypes = [_vp, _i64, _vp, _vp]
        L.rsvd_plan_postselect.restype = ctypes.c_int
        L.rsvd_plan_tiles.argtypes = [_vp, _vp, _i64, _vp]
        L.rsvd_plan_tiles.restype = ctypes.c_int
        L.rsvd_plan_set_tiles.argtypes = [_vp, _vp, _i64]
        L.rsvd_plan_set_tiles.restype = ctypes.c_int
        L.rsvd_plan_workspace_bytes.argtypes = [_vp]
        L.rsvd_plan_workspace_bytes.restype = _i64
        L.rsvd_plan_destroy.argtypes = [_vp]
        L.rsvd_plan_destroy.restype = None
        L.rsvd_last_error.argtypes = []
        L.rsvd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status):
    if status != RSVD_OK:
        raise RsvdError(status, lib().rsvd_last_error().decode(errors="replace"))
    return status


def ptr_array(ptrs):
    arr = (_vp * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr
