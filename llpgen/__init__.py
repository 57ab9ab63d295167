"""Seeded synthetic inputs for the LLP sweep (shared by the oracle tests, the GPU
tests and the benchmark).

The generators draw random numbers and lay inputs out; they contain none of the
method's arithmetic (no forbidden test, no advance, no fixpoint).  All draws come
from counter-based splitmix64 streams, so every array is a pure function of its
parameters and seed, independent of thread count.  The C source is
``llpgen/llpgen.c``; ``build()`` compiles it with gcc.

Workload recipes (sizes and value ranges follow the evaluation configurations):

* ``uniform_graph``  - n vertices, m_rand arcs with u ~ U[0,n), v uniform over the
  other n-1 vertices, plus a Hamiltonian cycle i -> i+1 mod n; weights U[lo,hi].
* ``rmat_graph``     - R-MAT (a,b,c,d) arcs, seeded vertex relabelling, then the
  Hamiltonian cycle; self-loops and duplicate arcs are kept.
* ``grid_graph``     - rows x cols 4-neighbour grid, both directions, per-arc weights.
* ``sm_prefs``       - independent uniform preference permutations (int16).
* ``job_dag``        - job j has min(Poisson(lam), j) distinct parents in [0, j).
* ``knapsack``       - items U[16,256], W U[256,4096], w U[1,W/4], v U[1,1000].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "llpgen.c")
_LIB = os.path.join(_HERE, "libllpgen.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i16p = ctypes.POINTER(ctypes.c_int16)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build() -> str:
    """Compile libllpgen.so in-tree (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.llpgen_mix64.restype = u64
    lib.llpgen_mix64.argtypes = [u64]
    lib.llpgen_key.restype = u64
    lib.llpgen_key.argtypes = [u64, u64]
    lib.llpgen_draw.restype = u64
    lib.llpgen_draw.argtypes = [u64, u64]
    lib.llpgen_uniform.argtypes = [i32, i64, i32, i32, i32, u64, _i32p, _i32p, _i32p]
    lib.llpgen_perm.argtypes = [i64, u64, u64, _i32p]
    lib.llpgen_rmat.argtypes = [i32, i32, dbl, dbl, dbl, i32, i32, i32, i32, u64, _i32p, _i32p, _i32p]
    lib.llpgen_grid_arcs.restype = i64
    lib.llpgen_grid_arcs.argtypes = [i32, i32]
    lib.llpgen_grid.argtypes = [i32, i32, i32, i32, u64, _i32p, _i32p, _i32p]
    lib.llpgen_sm.argtypes = [i32, u64, _i16p, _i16p]
    lib.llpgen_dag.argtypes = [i32, dbl, i32, i32, u64, _i32p, _i32p, _i32p]
    lib.llpgen_knapsack.argtypes = [u64, i64, i32, i32, i32, i32, i32, _i32p, _i32p, _i32p]
    lib.llpgen_u64.argtypes = [i64, u64, _u64p]
    lib.llpgen_csr.argtypes = [i32, i64, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p]
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(_i32p) if a is not None else None


def mix64(z: int) -> int:
    return int(_load().llpgen_mix64(z))


def draw(seed: int, tag: int, i: int) -> int:
    lib = _load()
    return int(lib.llpgen_draw(lib.llpgen_key(seed, tag), i))


# ---------------------------------------------------------------- graphs
class EdgeList:
    """Directed arcs (src[e] -> dst[e], weight w[e]) over n vertices."""

    def __init__(self, n, src, dst, w):
        self.n = int(n)
        self.src = src
        self.dst = dst
        self.w = w

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def uniform_graph(n: int, m_rand: int, wlo: int = 1, whi: int = 100, seed: int = 1,
                  cycle: bool = True) -> EdgeList:
    m = m_rand + (n if cycle else 0)
    src = np.empty(m, np.int32); dst = np.empty(m, np.int32); w = np.empty(m, np.int32)
    _load().llpgen_uniform(n, m_rand, int(cycle), wlo, whi, seed, _p32(src), _p32(dst), _p32(w))
    return EdgeList(n, src, dst, w)


def rmat_graph(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
               wlo: int = 1, whi: int = 255, seed: int = 22, relabel: bool = True,
               cycle: bool = True) -> EdgeList:
    n = 1 << scale
    m = n * ef + (n if cycle else 0)
    src = np.empty(m, np.int32); dst = np.empty(m, np.int32); w = np.empty(m, np.int32)
    _load().llpgen_rmat(scale, ef, a, b, c, int(relabel), int(cycle), wlo, whi, seed,
                        _p32(src), _p32(dst), _p32(w))
    return EdgeList(n, src, dst, w)


def grid_graph(rows: int, cols: int, wlo: int = 1, whi: int = 1000, seed: int = 100) -> EdgeList:
    lib = _load()
    m = int(lib.llpgen_grid_arcs(rows, cols))
    src = np.empty(m, np.int32); dst = np.empty(m, np.int32); w = np.empty(m, np.int32)
    lib.llpgen_grid(rows, cols, wlo, whi, seed, _p32(src), _p32(dst), _p32(w))
    return EdgeList(rows * cols, src, dst, w)


def csr(n: int, key, a, b=None):
    """Stable counting sort by key: returns (ptr[n+1], a_sorted, b_sorted|None)."""
    m = int(key.shape[0])
    key = np.ascontiguousarray(key, np.int32)
    a = np.ascontiguousarray(a, np.int32)
    ptr = np.empty(n + 1, np.int32)
    a_out = np.empty(m, np.int32)
    b_out = None
    if b is not None:
        b = np.ascontiguousarray(b, np.int32)
        b_out = np.empty(m, np.int32)
    _load().llpgen_csr(n, m, _p32(key), _p32(a), _p32(b), _p32(ptr), _p32(a_out), _p32(b_out))
    return ptr, a_out, b_out


class CSRGraph:
    """In-CSR (sorted by destination: in_ptr, in_src, in_w) and out-CSR (sorted by
    source: out_ptr, out_dst, out_w) of an EdgeList; arcs keep their input order
    inside each row."""

    def __init__(self, g: EdgeList, weighted: bool = True, out_weights: bool = False):
        self.n, self.m = g.n, g.m
        self.in_ptr, self.in_src, self.in_w = csr(g.n, g.dst, g.src, g.w if weighted else None)
        self.out_ptr, self.out_dst, self.out_w = csr(g.n, g.src, g.dst,
                                                     g.w if (weighted and out_weights) else None)


def max_outdeg_source(g: EdgeList) -> int:
    """Vertex of highest out-degree, smallest id on ties."""
    deg = np.bincount(g.src, minlength=g.n)
    return int(np.argmax(deg))


# ---------------------------------------------------------------- stable marriage
def sm_prefs(n: int, seed: int = 3):
    """(mpref, wrank) int16 [n, n]: mpref[m, i] = i-th woman on man m's list;
    wrank[w, m] = rank of man m on woman w's list (0 = most preferred)."""
    assert n <= 32767
    mpref = np.empty((n, n), np.int16)
    wrank = np.empty((n, n), np.int16)
    _load().llpgen_sm(n, seed, mpref.ctypes.data_as(_i16p), wrank.ctypes.data_as(_i16p))
    return mpref, wrank


# ---------------------------------------------------------------- jobs
def job_dag(n: int, lam: float = 8.0, dlo: int = 1, dhi: int = 1000, seed: int = 4):
    """(pred_ptr[n+1], pred_idx[E], dur[n]) int32."""
    lib = _load()
    pred_ptr = np.empty(n + 1, np.int32)
    lib.llpgen_dag(n, lam, dlo, dhi, seed, _p32(pred_ptr), None, None)
    pred_idx = np.empty(int(pred_ptr[-1]), np.int32)
    dur = np.empty(n, np.int32)
    lib.llpgen_dag(n, lam, dlo, dhi, seed, _p32(pred_ptr), _p32(pred_idx), _p32(dur))
    return pred_ptr, pred_idx, dur


# ---------------------------------------------------------------- knapsack
def knapsack(inst: int, seed: int = 5, nlo: int = 16, nhi: int = 256, Wlo: int = 256,
             Whi: int = 4096, vmax: int = 1000):
    """(wt[items], val[items], W) for instance number inst of a seeded family."""
    lib = _load()
    hdr = np.empty(2, np.int32)
    lib.llpgen_knapsack(seed, inst, nlo, nhi, Wlo, Whi, vmax, _p32(hdr), None, None)
    items, W = int(hdr[0]), int(hdr[1])
    wt = np.empty(items, np.int32); val = np.empty(items, np.int32)
    lib.llpgen_knapsack(seed, inst, nlo, nhi, Wlo, Whi, vmax, _p32(hdr), _p32(wt), _p32(val))
    return wt, val, W


# ---------------------------------------------------------------- reduction
def u64_words(n: int, seed: int = 7):
    x = np.empty(n, np.uint64)
    _load().llpgen_u64(n, seed, x.ctypes.data_as(_u64p))
    return x


# ---------------------------------------------------------------- helpers
def permutation(n: int, seed: int, tag: int = 0x99):
    p = np.empty(n, np.int32)
    _load().llpgen_perm(n, seed, tag, _p32(p))
    return p


def uniform_ints(n: int, lo: int, hi: int, seed: int, tag: int = 0x98):
    """n integers U[lo, hi] (vectorised from the splitmix64 stream)."""
    lib = _load()
    key = int(lib.llpgen_key(seed, tag))
    i = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    span = np.uint64(hi - lo + 1)
    return (np.int64(lo) + (((z >> np.uint64(32)) * span) >> np.uint64(32)).astype(np.int64)).astype(np.int64)


def job_succ(pred_ptr, pred_idx):
    """Successor lists (succ_ptr[n+1], succ_idx[E]) holding the same arcs as the
    predecessor lists, grouped by predecessor (stable)."""
    n = int(pred_ptr.shape[0]) - 1
    child = np.repeat(np.arange(n, dtype=np.int32), np.diff(pred_ptr).astype(np.int64))
    ptr, idx, _ = csr(n, pred_idx, child)
    return ptr, idx


# ---------------------------------------------------------------- batch workload
def batch_workload(n_knap: int = 4096, n_sssp: int = 4096, seed: int = 5, sssp_nlo: int = 256,
                   sssp_nhi: int = 4096, deg: int = 8):
    """Mixed batch: n_knap knapsack instances of the seeded family and n_sssp
    small SSSP graphs (n U[sssp_nlo, sssp_nhi], deg*n uniform arcs without
    self-loops plus the Hamiltonian cycle, w U[1,100], source 0), interleaved
    by a seeded permutation.  Returns a list of tuples
    ("knapsack", wt, val, W) / ("sssp", EdgeList, source)."""
    items = [("knapsack",) + tuple(knapsack(i, seed=seed)) for i in range(n_knap)]
    ns = uniform_ints(n_sssp, sssp_nlo, sssp_nhi, seed, tag=0x97) if n_sssp else []
    for i in range(n_sssp):
        n = int(ns[i])
        g = uniform_graph(n, deg * n, 1, 100, seed=(seed << 24) + i)
        items.append(("sssp", g, 0))
    order = permutation(len(items), seed, tag=0x96) if items else []
    return [items[int(k)] for k in order]

