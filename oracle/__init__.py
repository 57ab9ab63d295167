"""CPU oracle for the LLP sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never imports,
loads or calls it; the two share no code.

``oracle/oracle.c`` holds plain sequential implementations of Algorithm LLP
(paper, Background section) for every plugin, in the natural value domain with
64-bit arithmetic.  This module builds it with gcc and wraps it with ctypes over
numpy arrays.  ``oracle/mlp.py`` holds the float64 reference of the learned
scheduler's network.

Status codes: 0 ok, 1 bad argument, 2 bad input, 3 infeasible, 4 overflow,
5 not converged, 8 cycle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

INF32 = 2**31 - 1
OK, E_ARG, E_INPUT, E_INFEASIBLE, E_OVERFLOW, E_NOT_CONVERGED, E_CYCLE = 0, 1, 2, 3, 4, 5, 8

_i32p = ctypes.POINTER(ctypes.c_int32)
_i16p = ctypes.POINTER(ctypes.c_int16)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build() -> str:
    """Compile liboracle.so in-tree (single-threaded, -O2); always recompiles."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-std=c11", "-Wall", _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_sssp_cyclic.argtypes = [i32, i64, _i32p, _i32p, _i32p, i32, i64, _i32p, i32, _i32p, _i64p]
    lib.oracle_sssp_bag.argtypes = [i32, i64, _i32p, _i32p, _i32p, i32, _i32p, _i64p]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_sssp_bag_timed.argtypes = [i32, i64, _i32p, _i32p, _i32p, i32, _i32p, _i64p, dp]
    lib.oracle_dijkstra_timed.argtypes = [i32, i64, _i32p, _i32p, _i32p, i32, _i32p, dp]
    lib.oracle_bfs_queue_timed.argtypes = [i32, i64, _i32p, _i32p, i32, _i32p, dp]
    lib.oracle_sm_scan.argtypes = [i32, _i16p, _i16p, i64, _i32p, _i32p, _i64p]
    lib.oracle_sm_bag.argtypes = [i32, _i16p, _i16p, _i32p, _i32p, _i64p]
    lib.oracle_jobs_cyclic.argtypes = [i32, _i32p, _i32p, _i32p, i64, _i32p, _i64p]
    lib.oracle_jobs_bag.argtypes = [i32, _i32p, _i32p, _i32p, _i32p]
    lib.oracle_knapsack.argtypes = [i32, i32, _i32p, _i32p, i64, _i32p, _i32p, _i64p]
    lib.oracle_tc.argtypes = [i32, i64, _i32p, _i32p, _u32p, _i64p]
    lib.oracle_reduce.restype = ctypes.c_uint64
    lib.oracle_reduce.argtypes = [i64, _u64p]
    _lib = lib
    return lib


def _c32(a):
    return None if a is None else np.ascontiguousarray(a, np.int32)


def _p(a, t=_i32p):
    return None if a is None else a.ctypes.data_as(t)


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _ret(status, what, value, check):
    if check and status != OK:
        raise OracleError(status, what)
    return value if check else (status, value)


# ------------------------------------------------------------------ SSSP / BFS
def sssp(n, src, dst, w, source, *, bag=False, max_passes=0, order=None, jacobi=False,
         check=True, info=None):
    """Shortest distances (int32; unreachable = 2**31-1).  w=None gives BFS levels."""
    src, dst, w, order = _c32(src), _c32(dst), _c32(w), _c32(order)
    out = np.empty(n, np.int32)
    cnt = ctypes.c_int64(0)
    lib = _load()
    if bag:
        st = lib.oracle_sssp_bag(n, src.shape[0], _p(src), _p(dst), _p(w), source, _p(out),
                                 ctypes.byref(cnt))
    else:
        st = lib.oracle_sssp_cyclic(n, src.shape[0], _p(src), _p(dst), _p(w), source, max_passes,
                                    _p(order), int(jacobi), _p(out), ctypes.byref(cnt))
    if info is not None:
        info["count"] = cnt.value
    return _ret(st, "sssp", out, check)


def bfs(n, src, dst, source, **kw):
    return sssp(n, src, dst, None, source, **kw)


def sssp_bag_timed(n, src, dst, w, source, check=True):
    """(distances, seconds): the FIFO-bag oracle with the time of the solve
    alone (its adjacency lists are built before the clock starts).  w=None
    gives BFS levels."""
    src, dst, w = _c32(src), _c32(dst), _c32(w)
    out = np.empty(n, np.int32)
    cnt, t = ctypes.c_int64(0), ctypes.c_double(0.0)
    st = _load().oracle_sssp_bag_timed(n, src.shape[0], _p(src), _p(dst), _p(w), source, _p(out),
                                       ctypes.byref(cnt), ctypes.byref(t))
    return _ret(st, "sssp", out, check), t.value


def dijkstra_timed(n, src, dst, w, source, check=True):
    """(distances, seconds): binary-heap Dijkstra (a textbook cross-check, not
    LLP); w=None gives unit weights."""
    src, dst, w = _c32(src), _c32(dst), _c32(w)
    out = np.empty(n, np.int32)
    t = ctypes.c_double(0.0)
    st = _load().oracle_dijkstra_timed(n, src.shape[0], _p(src), _p(dst), _p(w), source, _p(out),
                                       ctypes.byref(t))
    return _ret(st, "dijkstra", out, check), t.value


def bfs_queue_timed(n, src, dst, source, check=True):
    """(levels, seconds): FIFO-queue BFS (a textbook cross-check, not LLP)."""
    src, dst = _c32(src), _c32(dst)
    out = np.empty(n, np.int32)
    t = ctypes.c_double(0.0)
    st = _load().oracle_bfs_queue_timed(n, src.shape[0], _p(src), _p(dst), source, _p(out), ctypes.byref(t))
    return _ret(st, "bfs", out, check), t.value


# ------------------------------------------------------------------ stable marriage
def stable_marriage(mpref, wrank, *, scan=False, max_passes=0, check=True, info=None):
    """(wife[n], proposal_index[n]) of the man-optimal stable matching."""
    n = mpref.shape[0]
    mpref = np.ascontiguousarray(mpref, np.int16)
    wrank = np.ascontiguousarray(wrank, np.int16)
    wife = np.empty(n, np.int32)
    prop = np.empty(n, np.int32)
    cnt = ctypes.c_int64(0)
    lib = _load()
    if scan:
        st = lib.oracle_sm_scan(n, _p(mpref, _i16p), _p(wrank, _i16p), max_passes, _p(wife), _p(prop),
                                ctypes.byref(cnt))
    else:
        st = lib.oracle_sm_bag(n, _p(mpref, _i16p), _p(wrank, _i16p), _p(wife), _p(prop),
                               ctypes.byref(cnt))
    if info is not None:
        info["count"] = cnt.value
    return _ret(st, "stable_marriage", (wife, prop), check)


# ------------------------------------------------------------------ jobs
def jobs(pred_ptr, pred_idx, dur, *, bag=False, max_passes=0, check=True, info=None):
    """Earliest start times (int32)."""
    pred_ptr, pred_idx, dur = _c32(pred_ptr), _c32(pred_idx), _c32(dur)
    n = dur.shape[0]
    out = np.empty(n, np.int32)
    lib = _load()
    if bag:
        st = lib.oracle_jobs_bag(n, _p(pred_ptr), _p(pred_idx), _p(dur), _p(out))
    else:
        cnt = ctypes.c_int64(0)
        st = lib.oracle_jobs_cyclic(n, _p(pred_ptr), _p(pred_idx), _p(dur), max_passes, _p(out),
                                    ctypes.byref(cnt))
        if info is not None:
            info["count"] = cnt.value
    return _ret(st, "jobs", out, check)


# ------------------------------------------------------------------ knapsack
def knapsack(wt, val, W, *, row=False, max_passes=0, check=True, info=None):
    """Best value (int); with row=True also the last DP row G[n][0..W]."""
    wt, val = _c32(wt), _c32(val)
    best = np.zeros(1, np.int32)
    last = np.empty(W + 1, np.int32) if row else None
    cnt = ctypes.c_int64(0)
    st = _load().oracle_knapsack(wt.shape[0], W, _p(wt), _p(val), max_passes, _p(best), _p(last),
                                 ctypes.byref(cnt))
    if info is not None:
        info["count"] = cnt.value
    value = (int(best[0]), last) if row else int(best[0])
    return _ret(st, "knapsack", value, check)


# ------------------------------------------------------------------ transitive closure
def transitive_closure(n, src, dst, *, check=True, info=None):
    """Reachability bit rows uint32[n, ceil(n/32)] (paths of length >= 1)."""
    src, dst = _c32(src), _c32(dst)
    words = (n + 31) // 32
    out = np.zeros((n, words), np.uint32)
    cnt = ctypes.c_int64(0)
    st = _load().oracle_tc(n, src.shape[0], _p(src), _p(dst), _p(out, _u32p), ctypes.byref(cnt))
    if info is not None:
        info["count"] = cnt.value
    return _ret(st, "transitive_closure", out, check)


# ------------------------------------------------------------------ reduction
def reduce_sum(x) -> int:
    """Sum of uint64 words modulo 2**64."""
    x = np.ascontiguousarray(x, np.uint64)
    return int(_load().oracle_reduce(x.shape[0], _p(x, _u64p)))
