"""ctypes loader for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never imports this package.

All functions take and return numpy float64 arrays (row-major).  Status
codes mirror the C file: 0 ok, -1 invalid argument, -2 allocation failure,
-4 non-finite input, -5 Jacobi did not converge.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

OK, ERR_INVALID, ERR_ALLOC, ERR_NONFINITE, ERR_NOCONV = 0, -1, -2, -4, -5

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_omega_entry.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_omega_entry.restype = ctypes.c_double
        L.orc_gaussian.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _dp]
        L.orc_gaussian.restype = None
        L.orc_hqr.argtypes = [ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp]
        L.orc_hqr.restype = ctypes.c_int
        L.orc_jacobi_cols.argtypes = [ctypes.c_int64, ctypes.c_int64, _dp, _dp,
                                      ctypes.c_int, _ip]
        L.orc_jacobi_cols.restype = ctypes.c_int
        L.orc_rsvd.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_uint64, ctypes.c_double, _dp, ctypes.c_int64,
                               _dp, _dp, ctypes.c_int64, _dp, _i64p, _dp, _dp, _i64p, _ip]
        L.orc_rsvd.restype = ctypes.c_int
        L.orc_fullsvd.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_double, _dp, ctypes.c_int64,
                                  _dp, _dp, ctypes.c_int64, _dp, _i64p, _dp, _ip]
        L.orc_fullsvd.restype = ctypes.c_int
        L.orc_rsvd_backward.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                        ctypes.c_double, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.orc_rsvd_backward.restype = ctypes.c_int
        L.orc_fullsvd_backward.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp,
                                           ctypes.c_double, _dp]
        L.orc_fullsvd_backward.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(_u32p), k.ctypes.data_as(_u32p),
                            out.ctypes.data_as(_u32p))
    return out


def gaussian(seed, n, l):
    om = np.empty((n, l), dtype=np.float64)
    lib().orc_gaussian(ctypes.c_uint64(seed), n, l, _ptr(om))
    return om


def hqr(Y):
    Y = _f64(Y)
    m, l = Y.shape
    Q = np.empty((m, l)); R = np.empty((l, l))
    st = lib().orc_hqr(m, l, _ptr(Y), _ptr(Q), _ptr(R))
    if st != OK:
        raise RuntimeError(f"orc_hqr status {st}")
    return Q, R


def jacobi_cols(G, max_sweeps=60):
    """One-sided Jacobi on the columns of G: returns (G J, J, status, sweeps)."""
    G = _f64(G).copy()
    r, c = G.shape
    J = np.empty((c, c))
    sw = ctypes.c_int(0)
    st = lib().orc_jacobi_cols(r, c, _ptr(G), _ptr(J), max_sweeps, ctypes.byref(sw))
    return G, J, st, sw.value


class Result:
    """U (m x k), S (k), VT (k x n), discarded weight w, k_kept, status, extras."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def rsvd(A, k, p, q, seed, delta=0.0):
    A = _f64(A)
    m, n = A.shape
    kk = min(k, m, n)
    l = min(kk + p, m, n)
    U = np.empty((m, kk)); S = np.empty(kk); VT = np.empty((kk, n))
    w = ctypes.c_double(0.0); kk_out = ctypes.c_int64(0)
    sig = np.empty(l); Qo = np.empty((m, l)); lo = ctypes.c_int64(0); sw = ctypes.c_int(0)
    st = lib().orc_rsvd(_ptr(A), m, n, n, k, p, q, ctypes.c_uint64(seed), delta,
                        _ptr(U), kk, _ptr(S), _ptr(VT), n, ctypes.byref(w),
                        ctypes.byref(kk_out), _ptr(sig), _ptr(Qo), ctypes.byref(lo),
                        ctypes.byref(sw))
    return Result(U=U, S=S, VT=VT, w=w.value, k_kept=kk_out.value, status=st,
                  sig_all=sig, Q=Qo, l=lo.value, sweeps=sw.value)


def fullsvd(A, k, delta=0.0):
    A = _f64(A)
    m, n = A.shape
    kk = min(k, m, n)
    U = np.empty((m, kk)); S = np.empty(kk); VT = np.empty((kk, n))
    w = ctypes.c_double(0.0); kk_out = ctypes.c_int64(0)
    sig = np.empty(min(m, n)); sw = ctypes.c_int(0)
    st = lib().orc_fullsvd(_ptr(A), m, n, n, k, delta, _ptr(U), kk, _ptr(S), _ptr(VT),
                           n, ctypes.byref(w), ctypes.byref(kk_out), _ptr(sig),
                           ctypes.byref(sw))
    return Result(U=U, S=S, VT=VT, w=w.value, k_kept=kk_out.value, status=st,
                  sig_all=sig, sweeps=sw.value)


def rsvd_backward(A, k, p, q, seed, dU, dS, dVT, delta=0.0, broad=0.0):
    """dA for L = <dU, U> + <dS, S> + <dVT, VT> of rsvd(A, k, p, q, seed, delta)."""
    A = _f64(A)
    m, n = A.shape
    dA = np.empty((m, n))
    st = lib().orc_rsvd_backward(_ptr(A), m, n, n, k, p, q, ctypes.c_uint64(seed), delta,
                                 _ptr(_f64(dU)), _ptr(_f64(dS)), _ptr(_f64(dVT)), broad, _ptr(dA))
    if st != OK:
        raise RuntimeError(f"orc_rsvd_backward status {st}")
    return dA


def fullsvd_backward(A, k, dU, dS, dVT, delta=0.0, broad=0.0):
    """dA of the same loss for the exact truncated SVD (reference gradient)."""
    A = _f64(A)
    m, n = A.shape
    dA = np.empty((m, n))
    st = lib().orc_fullsvd_backward(_ptr(A), m, n, n, k, delta, _ptr(_f64(dU)), _ptr(_f64(dS)),
                                    _ptr(_f64(dVT)), broad, _ptr(dA))
    if st != OK:
        raise RuntimeError(f"orc_fullsvd_backward status {st}")
    return dA


def postselect(S_list, k_kept, chi):
    """Sector post-selection (Sec. III.A): after one truncation per symmetry
    sector, keep the chi largest singular values over all sectors.  S_list[b]
    holds sector b's values (its first k_kept[b] are the candidates).  The
    candidates are ranked by value descending, then sector ascending, then
    index ascending, and the first chi are kept.  Returns the number kept per
    sector.  Written as the definition: a full sort of all candidates."""
    cand = []
    for b, (S, kk) in enumerate(zip(S_list, k_kept)):
        for j in range(int(kk)):
            cand.append((-float(S[j]), b, j))
    cand.sort()
    chi_s = [0] * len(S_list)
    for _, b, _ in cand[:max(0, int(chi))]:
        chi_s[b] += 1
    return chi_s


def rsvd_adaptive(A, k0, k_max, p, q, seed, delta):
    """Fixed-error RSVD with an adaptive rank (the outlook of Sec. V): the
    RSVD of rank k = k0, 2 k0, 4 k0, ... (capped at min(k_max, m, n)) with one
    seed, until the relative discarded-weight cut delta binds inside the
    sketch (k_kept < k) or the cap is reached.  Returns (result, attempts)."""
    A = _f64(A)
    kcap = min(k_max, *A.shape)
    k = min(k0, kcap)
    attempts = 0
    while True:
        res = rsvd(A, k, p, q, seed, delta)
        attempts += 1
        if res.status != OK or res.k_kept < k or k >= kcap:
            return res, attempts
        k = min(2 * k, kcap)
