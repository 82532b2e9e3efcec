"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Every function here is the plain definition of the join (Sections III.A,
III.C, IV.C and VI.E of the paper), computed by ``ejoin_oracle.c`` with the
canonical FP64 rule documented there:

    sim64(r, s) = dot(r, s) / sqrt(dot(r, r) * dot(s, s)),  0 for a zero row,
    dots summed sequentially over k = 0..d-1 without fused multiply-add.

Inputs are row-major float32 arrays of shape (n, ld) with ld >= d; only the
first d columns are read.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libejoin_oracle.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        fp = C.POINTER(C.c_float)
        i64 = C.c_int64
        L.eo_sim64.restype = C.c_double
        L.eo_sim64.argtypes = [fp, fp, C.c_int]
        L.eo_sim64_pairs.restype = C.c_int
        L.eo_sim64_pairs.argtypes = [fp, i64, fp, i64, C.c_int,
                                     C.POINTER(i64), C.POINTER(i64), i64,
                                     C.POINTER(C.c_double), C.c_int]
        L.eo_threshold.restype = i64
        L.eo_threshold.argtypes = [fp, i64, i64, fp, i64, i64, C.c_int, C.c_double,
                                   C.c_int, C.c_double,
                                   C.POINTER(C.POINTER(C.c_int32)),
                                   C.POINTER(C.POINTER(C.c_int32)),
                                   C.POINTER(C.POINTER(C.c_double)),
                                   C.POINTER(i64)]
        L.eo_topk.restype = C.c_int
        L.eo_topk.argtypes = [fp, i64, i64, fp, i64, i64, C.c_int, C.c_int, C.c_int,
                              C.POINTER(i64), C.POINTER(C.c_double)]
        L.eo_sim_matrix.restype = C.c_int
        L.eo_sim_matrix.argtypes = [fp, i64, i64, fp, i64, i64, C.c_int, C.c_int,
                                    C.POINTER(C.c_double)]
        L.eo_free.restype = None
        L.eo_free.argtypes = [C.c_void_p]
        L.eo_max_threads.restype = C.c_int
        L.eo_max_threads.argtypes = []
        _lib = L
    return _lib


class OracleError(ValueError):
    pass


def _prep(X, d):
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise OracleError("expected a 2-D array")
    n, ld = X.shape
    if d is None:
        d = ld
    if d > ld or d < 1:
        raise OracleError("need 1 <= d <= ld")
    return X, n, ld, d


def _fptr(X):
    return X.ctypes.data_as(C.POINTER(C.c_float))


def max_threads() -> int:
    return int(lib().eo_max_threads())


def sim64(r, s) -> float:
    """Canonical similarity of two 1-D float32 vectors of equal length."""
    r = np.ascontiguousarray(r, dtype=np.float32).ravel()
    s = np.ascontiguousarray(s, dtype=np.float32).ravel()
    if r.shape != s.shape:
        raise OracleError("length mismatch")
    return float(lib().eo_sim64(_fptr(r), _fptr(s), r.size))


def sim64_pairs(R, S, ri, si, d=None, threads: int = 0) -> np.ndarray:
    """sim64(R[ri[p]], S[si[p]]) for each p."""
    R, nR, ldR, d = _prep(R, d)
    S, nS, ldS, d2 = _prep(S, d)
    ri = np.ascontiguousarray(ri, dtype=np.int64)
    si = np.ascontiguousarray(si, dtype=np.int64)
    if ri.shape != si.shape:
        raise OracleError("index arrays differ in length")
    if ri.size and (ri.min() < 0 or ri.max() >= nR or si.min() < 0 or si.max() >= nS):
        raise OracleError("pair index out of range")
    out = np.empty(ri.size, dtype=np.float64)
    lib().eo_sim64_pairs(_fptr(R), ldR, _fptr(S), ldS, d,
                         ri.ctypes.data_as(C.POINTER(C.c_int64)),
                         si.ctypes.data_as(C.POINTER(C.c_int64)), ri.size,
                         out.ctypes.data_as(C.POINTER(C.c_double)), threads)
    return out


def sim_matrix(R, S, d=None, threads: int = 0) -> np.ndarray:
    """Dense (|R|, |S|) matrix of sim64 values (small inputs only)."""
    R, nR, ldR, d = _prep(R, d)
    S, nS, ldS, _ = _prep(S, d)
    out = np.empty((nR, nS), dtype=np.float64)
    rc = lib().eo_sim_matrix(_fptr(R), nR, ldR, _fptr(S), nS, ldS, d, threads,
                             out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise OracleError("allocation failure")
    return out


def threshold(R, S, theta: float, d=None, threads: int = 0, tie_eps: float = 1e-12):
    """All (i, j) with sim64(R_i, S_j) >= theta, sorted by (i, j).

    Returns (ri int32, si int32, score float64, n_ties)."""
    R, nR, ldR, d = _prep(R, d)
    S, nS, ldS, _ = _prep(S, d)
    if not np.isfinite(theta):
        raise OracleError("theta must be finite")
    pr = C.POINTER(C.c_int32)()
    ps = C.POINTER(C.c_int32)()
    pc = C.POINTER(C.c_double)()
    ties = C.c_int64(0)
    n = lib().eo_threshold(_fptr(R), nR, ldR, _fptr(S), nS, ldS, d, float(theta),
                           threads, float(tie_eps), C.byref(pr), C.byref(ps),
                           C.byref(pc), C.byref(ties))
    if n == -1:
        raise OracleError("non-finite input")
    if n < 0:
        raise OracleError("allocation failure")
    try:
        ri = np.ctypeslib.as_array(pr, shape=(max(n, 1),))[:n].copy()
        si = np.ctypeslib.as_array(ps, shape=(max(n, 1),))[:n].copy()
        sc = np.ctypeslib.as_array(pc, shape=(max(n, 1),))[:n].copy()
    finally:
        for p in (pr, ps, pc):
            lib().eo_free(C.cast(p, C.c_void_p))
    return ri, si, sc, int(ties.value)


def topk(R, S, k: int, d=None, threads: int = 0):
    """Per R row the first min(k, |S|) S indices ordered by (sim64 desc,
    index asc); missing slots are (-1, -inf).  Returns (idx int64 (|R|, k),
    score float64 (|R|, k))."""
    R, nR, ldR, d = _prep(R, d)
    S, nS, ldS, _ = _prep(S, d)
    if k < 1:
        raise OracleError("k must be >= 1")
    idx = np.empty((nR, k), dtype=np.int64)
    sc = np.empty((nR, k), dtype=np.float64)
    rc = lib().eo_topk(_fptr(R), nR, ldR, _fptr(S), nS, ldS, d, int(k), threads,
                       idx.ctypes.data_as(C.POINTER(C.c_int64)),
                       sc.ctypes.data_as(C.POINTER(C.c_double)))
    if rc == -1:
        raise OracleError("non-finite input")
    if rc != 0:
        raise OracleError("allocation failure")
    return idx, sc


def topk_range(R, S, k: int, theta: float, d=None, threads: int = 0):
    """The range predicate combined with the top-k condition (the range join
    with a k cap of the scan-versus-probe study, Section VI.E): per R row the
    first min(k, m) of the m S indices with sim64 >= theta, ordered by
    (sim64 desc, index asc); missing slots are (-1, -inf).  Written out from
    the two definitions above: the threshold join's pairs of each row, sorted.
    Returns (idx int64 (|R|, k), score float64 (|R|, k))."""
    R, nR, _, d = _prep(R, d)
    ri, si, sc, _ = threshold(R, S, theta, d=d, threads=threads)
    idx = np.full((nR, k), -1, dtype=np.int64)
    out = np.full((nR, k), -np.inf, dtype=np.float64)
    order = np.lexsort((si, -sc, ri))          # by row, then sim64 desc, then index
    ri, si, sc = ri[order], si[order], sc[order]
    starts = np.searchsorted(ri, np.arange(nR), side="left")
    ends = np.searchsorted(ri, np.arange(nR), side="right")
    for i in range(nR):
        m = min(k, ends[i] - starts[i])
        idx[i, :m] = si[starts[i]:starts[i] + m]
        out[i, :m] = sc[starts[i]:starts[i] + m]
    return idx, out
