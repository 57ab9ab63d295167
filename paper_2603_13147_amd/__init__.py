"""Python binding of libllp, the MI355X (gfx950) LLP sweep.

Argument marshalling only: every step of every solve runs in the HIP kernels
of ``libllp.so`` behind the C ABI declared in ``include/llp.h``.  Torch is used
for device memory (tensors) and streams.  There is no CPU fallback: importing
works without the library, but every call raises ``LLPError`` when
``libllp.so`` is missing or no GPU is present.

Build the library with ``__graft_entry__.build()`` (or ``python -m
paper_2603_13147_amd._build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libllp.so")

INF32 = 2**31 - 1

# status codes (llp_status)
OK, E_ARG, E_INPUT, E_INFEASIBLE, E_OVERFLOW, E_NOT_CONVERGED, E_WORKSPACE, E_HIP, E_CYCLE, E_ABORTED = range(10)

SCHED_PLAIN, SCHED_FIXED, SCHED_LEARNED, SCHED_HYBRID, SCHED_RANDOM, SCHED_SCRIPT = range(6)
MODE_PULL, MODE_DENSE, MODE_PUSH = 0, 1, 2
DCLASS_BASE, DCLASS_WIDE, DCLASS_NONE, DCLASS_EXPLICIT = 0, 1, 2, 3


def round_code(mode, dclass=DCLASS_NONE):
    return mode | (dclass << 8)
PUSH, DENSE, VALIDATE, ASYNC, VERIFY, TRACE, TIMING, JOBS_PULL = (1 << i for i in range(8))
KIND_SSSP, KIND_BFS, KIND_SM, KIND_JOBS, KIND_KNAPSACK, KIND_TC, KIND_REDUCE, KIND_BATCH = range(1, 9)

MLP_IN, MLP_HID, MLP_OUT = 12, 64, 5
MLP_PARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 5 * 64 + 5


class LLPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"llp status {status}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("edges_inspected", ctypes.c_int64), ("advances", ctypes.c_int64),
                ("expand_edges", ctypes.c_int64), ("eval_launches", ctypes.c_int64),
                ("device_ms", ctypes.c_float), ("kernel_ms", ctypes.c_float),
                ("push_edges", ctypes.c_int64), ("pre_launches", ctypes.c_int64),
                ("pre_ms", ctypes.c_float), ("pad", ctypes.c_float), ("states_gathered", ctypes.c_int64),
                ("bitmap_rounds", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TraceRec(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("mode", ctypes.c_int32), ("in_count", ctypes.c_int32),
                ("out_count", ctypes.c_int32), ("in_edges", ctypes.c_int64), ("out_edges", ctypes.c_int64),
                ("bucket", ctypes.c_int32), ("pending", ctypes.c_int32), ("bitmap", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


TRACE_DTYPE = np.dtype([("round", np.int32), ("mode", np.int32), ("in_count", np.int32),
                        ("out_count", np.int32), ("in_edges", np.int64), ("out_edges", np.int64),
                        ("bucket", np.int32), ("pending", np.int32), ("bitmap", np.int32),
                        ("pad", np.int32)])


class Opts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("sched", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("delta", ctypes.c_int32), ("max_rounds", ctypes.c_int64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p), ("warm_start", ctypes.c_void_p),
                ("status_dev", ctypes.c_void_p), ("abort_host", ctypes.c_void_p),
                ("stats", ctypes.POINTER(Stats)), ("chunk", ctypes.c_int32), ("block", ctypes.c_int32),
                ("trace_dev", ctypes.c_void_p), ("trace_cap", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("plan", ctypes.c_void_p), ("plan_len", ctypes.c_int64)]


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("in_ptr", ctypes.c_void_p), ("in_src", ctypes.c_void_p), ("in_w", ctypes.c_void_p),
                ("out_ptr", ctypes.c_void_p), ("out_dst", ctypes.c_void_p), ("out_w", ctypes.c_void_p)]


class Instance(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("cap_or_source", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("m", ctypes.c_int64), ("in_off", ctypes.c_int64),
                ("out_off", ctypes.c_int64)]


INSTANCE_DTYPE = np.dtype([("kind", np.int32), ("n", np.int32), ("cap_or_source", np.int32),
                           ("pad", np.int32), ("m", np.int64), ("in_off", np.int64), ("out_off", np.int64)])

_lib = None


def lib():
    """The loaded libllp.so (raises LLPError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LLPError(E_HIP, f"{LIB_PATH} is missing: build the HIP library first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    po = ctypes.POINTER(Opts)
    L.llp_workspace_bytes.restype = sz
    L.llp_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, po]
    L.llp_solve_sssp.argtypes = [ctypes.POINTER(Graph), i32, vp, po]
    L.llp_solve_bfs.argtypes = [ctypes.POINTER(Graph), i32, vp, po]
    L.llp_last_error.restype = ctypes.c_char_p
    L.llp_version.restype = ctypes.c_char_p
    L.llp_sched_set_weights.argtypes = [vp]
    for name, args in [
        ("llp_solve_sm", [i32, vp, vp, vp, vp, po]),
        ("llp_solve_jobs", [i32, vp, vp, vp, vp, vp, vp, po]),
        ("llp_solve_knapsack", [i32, i32, vp, vp, vp, vp, po]),
        ("llp_solve_tc", [i32, i64, vp, vp, vp, po]),
        ("llp_solve_reduce", [i64, vp, vp, po]),
        ("llp_solve_reduce_noalloc", [i64, vp, vp, po]),
        ("llp_solve_batch", [i32, vp, vp, i64, vp, i64, vp, po]),
        ("llp_solve_batch_graph", [i32, vp, vp, i64, vp, i64, vp, po]),
        ("llp_autotune_batch", [i32, vp, vp, i64, vp, i64, ctypes.c_char_p, sz, po]),
        ("llp_autotune_get", [ctypes.c_int, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        ("llp_autotune_graph", [ctypes.POINTER(Graph), i32, i32, vp, ctypes.c_char_p, sz, po]),
        ("llp_autotune_lookup", [i32, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        ("llp_autotune_save", [ctypes.c_char_p]),
        ("llp_autotune_load", [ctypes.c_char_p, ctypes.POINTER(i32)]),
        ("llp_mlp_forward", [i32, vp, vp, vp, vp, vp]),
        ("llp_mlp_loss", [i32, vp, vp, vp, vp, vp]),
        ("llp_mlp_backward", [i32, vp, vp, vp, vp, vp, vp]),
        ("llp_mlp_adam", [vp, vp, vp, vp, i32, ctypes.c_float, vp]),
        ("llp_trace_features", [i64, vp, i32, i64, i32, vp, vp]),
    ]:
        if hasattr(L, name):
            getattr(L, name).argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names of the entry points libllp.so exports (checked against include/llp.h)."""
    L = lib()
    return L


def _check(status):
    if status != OK:
        raise LLPError(status, lib().llp_last_error().decode(errors="replace"))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise LLPError(E_HIP, "no GPU visible: libllp runs only on an MI355X (gfx950)")
    return torch


def _dev(t, dtype):
    """Device tensor of the given torch dtype from a numpy array or tensor."""
    torch = _torch()
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device="cuda", dtype=dtype)
    return t.contiguous()


def _out(t, shape, dtype, name):
    """A caller-supplied output (or a new one when t is None): a contiguous GPU
    tensor of exactly this dtype and shape, since the kernels write it whole."""
    torch = _torch()
    shape = tuple(int(x) for x in shape)
    if t is None:
        return torch.empty(shape, dtype=dtype, device="cuda")
    _need(t, shape, dtype, name)
    return t


def _need(t, shape, dtype, name):
    """Rejects anything but a contiguous GPU tensor of this dtype and shape."""
    torch = _torch()
    ok = (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
          and tuple(t.shape) == tuple(shape))
    if not ok:
        got = (f"{t.dtype} {tuple(t.shape)} on {t.device}" if isinstance(t, torch.Tensor) else type(t).__name__)
        raise LLPError(E_ARG, f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, got {got}")


def _length(t, k, name):
    if t.dim() != 1 or int(t.shape[0]) != k:
        raise LLPError(E_ARG, f"{name} must be one-dimensional with {k} entries, got shape {tuple(t.shape)}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(sched=SCHED_PLAIN, flags=0, delta=0, max_rounds=0, workspace=None, stats=None, chunk=0,
              block=0, trace=None, seed=0, warm_start=None, abort_host=None, status_dev=None, plan=None):
    o = Opts()
    o.size = ctypes.sizeof(Opts)
    o.sched = sched
    o.flags = flags
    o.delta = delta
    o.max_rounds = max_rounds
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.stream = _stream()
    if warm_start is not None:
        o.warm_start = warm_start.data_ptr()
    if status_dev is not None:
        o.status_dev = status_dev.data_ptr()
    if abort_host is not None:
        o.abort_host = abort_host.data_ptr()
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    o.chunk = chunk
    o.block = block
    if trace is not None:
        o.trace_dev = trace.data_ptr()
        o.trace_cap = trace.numel() // ctypes.sizeof(TraceRec)
    o.seed = seed
    if plan is not None:
        o.plan = plan.data_ptr()
        o.plan_len = plan.numel()
    return o


def workspace(kind, n, m, chunk=0):
    """Device scratch for a solve of this kind and size (chunk: the launch knob
    the solve will be given, see llp_opts.chunk)."""
    torch = _torch()
    o = Opts()
    o.size = ctypes.sizeof(Opts)
    o.chunk = chunk
    nbytes = int(lib().llp_workspace_bytes(kind, n, m, ctypes.byref(o)))
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")


# ---------------------------------------------------------------- graphs
class DeviceGraph:
    """Device copy of a CSRGraph-like object (in_ptr/in_src/in_w, out_ptr/out_dst/out_w)."""

    def __init__(self, csr, weighted=True):
        torch = _torch()
        i32 = torch.int32
        self.n, self.m = int(csr.n), int(csr.m)
        self.in_ptr = _dev(csr.in_ptr, i32)
        self.in_src = _dev(csr.in_src, i32)
        self.in_w = _dev(csr.in_w, i32) if (weighted and csr.in_w is not None) else None
        self.out_ptr = _dev(csr.out_ptr, i32)
        self.out_dst = _dev(csr.out_dst, i32)
        ow = getattr(csr, "out_w", None)
        self.out_w = _dev(ow, i32) if (weighted and ow is not None) else None

    def cstruct(self):
        g = Graph()
        g.n, g.m = self.n, self.m
        g.in_ptr, g.in_src, g.in_w = (t.data_ptr() if t is not None else None
                                      for t in (self.in_ptr, self.in_src, self.in_w))
        g.out_ptr, g.out_dst, g.out_w = (t.data_ptr() if t is not None else None
                                         for t in (self.out_ptr, self.out_dst, self.out_w))
        return g


def _graph_solve(fn, kind, dg, source, out, opts):
    torch = _torch()
    out = _out(out, (dg.n,), torch.int32, "out")
    g = dg.cstruct()
    _check(fn(ctypes.byref(g), int(source), _ptr(out), ctypes.byref(opts)))
    return out


def sssp(dg, source, out=None, ws=None, **kw):
    """Shortest distances from `source` (int32 tensor; 2**31-1 = unreachable)."""
    if ws is None:
        ws = workspace(KIND_SSSP, dg.n, dg.m, kw.get("chunk", 0))
    o = make_opts(workspace=ws, **kw)
    return _graph_solve(lib().llp_solve_sssp, KIND_SSSP, dg, source, out, o)


def bfs(dg, source, out=None, ws=None, **kw):
    """Breadth-first levels from `source` (int32 tensor; 2**31-1 = unreachable)."""
    if ws is None:
        ws = workspace(KIND_BFS, dg.n, dg.m, kw.get("chunk", 0))
    o = make_opts(workspace=ws, **kw)
    return _graph_solve(lib().llp_solve_bfs, KIND_BFS, dg, source, out, o)


# ---------------------------------------------------------------- stable marriage
def stable_marriage(mpref, wrank, wife=None, prop=None, ws=None, **kw):
    """Man-optimal stable matching: (wife[n], proposal_index[n]) int32 tensors.
    mpref[m, i] = i-th woman on man m's list; wrank[w, m] = rank of m for w."""
    torch = _torch()
    mp = _dev(mpref, torch.int16)
    wr = _dev(wrank, torch.int16)
    n = int(mp.shape[0])
    if tuple(mp.shape) != (n, n) or tuple(wr.shape) != (n, n):
        raise LLPError(E_ARG, "mpref and wrank must both be n x n")
    wife = _out(wife, (n,), torch.int32, "wife")
    prop = _out(prop, (n,), torch.int32, "prop")
    if ws is None:
        ws = workspace(KIND_SM, n, 0)
    o = make_opts(workspace=ws, **kw)
    _check(lib().llp_solve_sm(n, _ptr(mp), _ptr(wr), _ptr(wife), _ptr(prop), ctypes.byref(o)))
    return wife, prop


# ---------------------------------------------------------------- jobs
def jobs(pred_ptr, pred_idx, dur, succ_ptr, succ_idx, out=None, ws=None, pull=False, **kw):
    """Earliest start times (int32 tensor) of the job DAG given by predecessor
    and successor lists; pull=True runs the pull form of the sweep."""
    torch = _torch()
    pp, pi, d = _dev(pred_ptr, torch.int32), _dev(pred_idx, torch.int32), _dev(dur, torch.int32)
    sp, si = _dev(succ_ptr, torch.int32), _dev(succ_idx, torch.int32)
    n = int(d.shape[0])
    _length(d, n, "dur")
    _length(pp, n + 1, "pred_ptr")
    _length(sp, n + 1, "succ_ptr")
    _length(si, int(pi.shape[0]), "succ_idx (one entry per predecessor arc)")
    out = _out(out, (n,), torch.int32, "out")
    if ws is None:
        ws = workspace(KIND_JOBS, n, int(pi.shape[0]))
    if pull:
        kw["flags"] = kw.get("flags", 0) | JOBS_PULL
    o = make_opts(workspace=ws, **kw)
    _check(lib().llp_solve_jobs(n, _ptr(pp), _ptr(pi), _ptr(d), _ptr(sp), _ptr(si), _ptr(out),
                                ctypes.byref(o)))
    return out


# ---------------------------------------------------------------- knapsack
def knapsack(wt, val, W, row=False, ws=None, **kw):
    """Best value of the 0-1 knapsack (int); with row=True also G[items][0..W]
    as an int32 tensor."""
    torch = _torch()
    w_, v_ = _dev(wt, torch.int32), _dev(val, torch.int32)
    items = int(w_.shape[0])
    _length(w_, items, "wt")
    _length(v_, items, "val")
    best = torch.zeros(1, dtype=torch.int32, device="cuda")
    last = torch.empty(W + 1, dtype=torch.int32, device="cuda") if row else None
    if ws is None:
        ws = workspace(KIND_KNAPSACK, items, W)
    o = make_opts(workspace=ws, **kw)
    _check(lib().llp_solve_knapsack(items, int(W), _ptr(w_), _ptr(v_), _ptr(best), _ptr(last),
                                    ctypes.byref(o)))
    return (int(best.item()), last) if row else int(best.item())


# ---------------------------------------------------------------- batch
class Batch:
    """Device-resident batch of independent instances for llp_solve_batch.

    items: tuples ("knapsack", wt, val, W) or ("sssp", graph, source) where
    graph has n, src, dst, w (an edge list; it is packed here as out-CSR
    grouped by tail, arcs in input order)."""

    def __init__(self, items):
        torch = _torch()
        desc = np.zeros(len(items), INSTANCE_DTYPE)
        chunks, pos, out = [], 0, 0
        self.out_slices = []
        for i, it in enumerate(items):
            if it[0] == "knapsack":
                _, wt, val, W = it
                wt = np.ascontiguousarray(wt, np.int32)
                val = np.ascontiguousarray(val, np.int32)
                desc[i] = (KIND_KNAPSACK, wt.shape[0], W, 0, 0, pos, out)
                chunks += [wt, val]
                pos += 2 * wt.shape[0]
                self.out_slices.append((out, 1))
                out += 1
            elif it[0] == "sssp":
                _, g, source = it
                n, m = int(g.n), int(g.src.shape[0])
                order = np.argsort(g.src, kind="stable")
                ptr = np.zeros(n + 1, np.int64)
                np.add.at(ptr, g.src.astype(np.int64) + 1, 1)
                ptr = np.cumsum(ptr).astype(np.int32)
                desc[i] = (KIND_SSSP, n, source, 0, m, pos, out)
                chunks += [ptr, g.dst[order].astype(np.int32), g.w[order].astype(np.int32)]
                pos += n + 1 + 2 * m
                self.out_slices.append((out, n))
                out += n
            else:
                raise LLPError(E_ARG, f"unknown instance kind {it[0]!r}")
        pool = np.concatenate(chunks) if chunks else np.zeros(1, np.int32)
        self.count = len(items)
        self.desc = torch.from_numpy(desc.view(np.uint8).copy()).cuda()
        self.pool = torch.from_numpy(pool.astype(np.int32)).cuda()
        self.pool_words = int(pos)
        self.out = torch.zeros(max(out, 1), dtype=torch.int32, device="cuda")
        self.out_words = int(out)
        self.status = torch.zeros(max(len(items), 1), dtype=torch.int32, device="cuda")
        self.ws = workspace(KIND_BATCH, 0, self.count)

    def _args(self):
        return (self.count, _ptr(self.desc), _ptr(self.pool), self.pool_words, _ptr(self.out),
                self.out_words, _ptr(self.status))

    def solve(self, graph=False, **kw):
        """Solve every instance (graph=True: replay a captured hipGraph)."""
        o = make_opts(workspace=kw.pop("ws", self.ws), **kw)
        fn = lib().llp_solve_batch_graph if graph else lib().llp_solve_batch
        _check(fn(*self._args(), ctypes.byref(o)))
        return self

    def autotune(self, **kw):
        """Time every launch shape on this batch; returns [(block, chunk, ms)]."""
        o = make_opts(workspace=kw.pop("ws", self.ws), **kw)
        buf = ctypes.create_string_buffer(4096)
        c, d, p, pw, out, ow, _ = self._args()
        _check(lib().llp_autotune_batch(c, d, p, pw, out, ow, buf, 4096, ctypes.byref(o)))
        rows = []
        for line in buf.value.decode().splitlines():
            b, ch, ms = line.split()
            rows.append((int(b), int(ch), float(ms)))
        return rows

    def results(self):
        """Per-instance results: int (knapsack best) or int32 array (SSSP dist)."""
        o = self.out.cpu().numpy()
        kinds = np.frombuffer(self.desc.cpu().numpy().tobytes(), INSTANCE_DTYPE)["kind"]
        return [int(o[a]) if kinds[i] == KIND_KNAPSACK else o[a:a + k].copy()
                for i, (a, k) in enumerate(self.out_slices)]


def autotune_get(kind=KIND_BATCH):
    """The most recently recorded (block, chunk) for kind on this device."""
    b, c = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().llp_autotune_get(kind, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def autotune_graph(dg, source, kind=KIND_SSSP, out=None, ws=None, **kw):
    """Time the sweep at 1..4 workgroups per CU on this graph and record the
    fastest for (kind, size class of m); returns ([(chunk, ms)], out)."""
    torch = _torch()
    if ws is None:
        ws = workspace(kind, dg.n, dg.m, 0)
    o = make_opts(workspace=ws, **kw)
    out = _out(out, (dg.n,), torch.int32, "out")
    g = dg.cstruct()
    buf = ctypes.create_string_buffer(1024)
    _check(lib().llp_autotune_graph(ctypes.byref(g), int(source), kind, _ptr(out), buf, 1024, ctypes.byref(o)))
    rows = []
    for line in buf.value.decode().splitlines():
        c, ms = line.split()
        rows.append((int(c), float(ms)))
    return rows, out


def autotune_lookup(kind, size):
    """(block, chunk) a solve of kind and size would take from the records."""
    b, c = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().llp_autotune_lookup(kind, int(size), ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def autotune_save(path):
    """Write every autotuner record to a JSON cache file."""
    _check(lib().llp_autotune_save(os.fsencode(path)))


def autotune_load(path):
    """Add the records of a JSON cache file; returns how many it held."""
    n = ctypes.c_int32(0)
    _check(lib().llp_autotune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


# ---------------------------------------------------------------- transitive closure / reduction
def transitive_closure(n, out_ptr, out_dst, ws=None, **kw):
    """Reachability bit rows (uint32 words as an int32 tensor [n, ceil(n/32)]):
    bit v & 31 of word v >> 5 in row u is set iff a path of length >= 1 leads
    from u to v."""
    torch = _torch()
    p, d = _dev(out_ptr, torch.int32), _dev(out_dst, torch.int32)
    _length(p, n + 1, "out_ptr")
    _length(d, int(d.shape[0]), "out_dst")
    words = (n + 31) // 32
    bits = torch.empty((n, words), dtype=torch.int32, device="cuda")
    if ws is None:
        ws = workspace(KIND_TC, n, int(d.shape[0]))
    o = make_opts(workspace=ws, **kw)
    _check(lib().llp_solve_tc(n, int(d.shape[0]), _ptr(p), _ptr(d), _ptr(bits), ctypes.byref(o)))
    return bits


def reduce_sum(x, ws=None, **kw):
    """Sum of uint64 words modulo 2**64 (x: numpy uint64 or an int64 tensor of the same bits)."""
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, np.uint64).view(np.int64))
    if x.dtype != torch.int64:
        raise LLPError(E_ARG, f"x must hold 64-bit words (int64 tensor or uint64 array), got {x.dtype}")
    x = x.to(device="cuda").contiguous()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    if ws is None:
        ws = workspace(KIND_REDUCE, x.numel(), 0)
    o = make_opts(workspace=ws, **kw)
    _check(lib().llp_solve_reduce(x.numel(), _ptr(x), _ptr(out), ctypes.byref(o)))
    return int(out.cpu().numpy().view(np.uint64)[0])


def reduce_sum_noalloc(x, out=None, **kw):
    """reduce_sum through llp_solve_reduce_noalloc: no device allocation by the
    library (x: an int64 CUDA tensor of the words' bits; out: optional int64[1]
    CUDA tensor for the result)."""
    torch = _torch()
    _need(x, (x.numel(),), torch.int64, "x")
    out = _out(out, (1,), torch.int64, "out")
    o = make_opts(**kw)
    _check(lib().llp_solve_reduce_noalloc(x.numel(), _ptr(x), _ptr(out), ctypes.byref(o)))
    return out


# ---------------------------------------------------------------- learned scheduler
def set_sched_weights(params):
    """Load FP32 master weights (LLP_MLP_PARAMS floats) for LLP_SCHED_LEARNED on the current device."""
    p = np.ascontiguousarray(np.asarray(params, np.float32).ravel())
    if p.shape[0] != MLP_PARAMS:
        raise LLPError(E_ARG, f"expected {MLP_PARAMS} parameters, got {p.shape[0]}")
    _torch()
    _check(lib().llp_sched_set_weights(p.ctypes.data_as(ctypes.c_void_p)))


def default_sched_weights_path():
    return os.path.join(_HERE, "sched_weights.npy")


def mlp_forward(params, x):
    """(logits[B,5] fp32, act[B,128] bf16 bits as int16) for device tensors params[5317], x[B,12]."""
    torch = _torch()
    B = int(x.shape[0])
    _need(params, (MLP_PARAMS,), torch.float32, "params")
    _need(x, (B, MLP_IN), torch.float32, "x")
    logits = torch.empty((B, MLP_OUT), dtype=torch.float32, device="cuda")
    act = torch.empty((B, 2 * MLP_HID), dtype=torch.int16, device="cuda")
    _check(lib().llp_mlp_forward(B, _ptr(params), _ptr(x), _ptr(logits), _ptr(act), _stream()))
    return logits, act


def mlp_loss(logits, labels):
    """(loss[1] fp32, dlogits[B,5]) for round-code labels[B] int32."""
    torch = _torch()
    B = int(logits.shape[0])
    _need(logits, (B, MLP_OUT), torch.float32, "logits")
    _need(labels, (B,), torch.int32, "labels")
    dl = torch.empty_like(logits)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().llp_mlp_loss(B, _ptr(logits), _ptr(labels), _ptr(dl), _ptr(loss), _stream()))
    return loss, dl


def mlp_backward(params, x, act, dlogits, grad):
    """grad += d loss / d params (grad: fp32[5317] device tensor)."""
    torch = _torch()
    B = int(x.shape[0])
    _need(params, (MLP_PARAMS,), torch.float32, "params")
    _need(x, (B, MLP_IN), torch.float32, "x")
    _need(act, (B, 2 * MLP_HID), torch.int16, "act")
    _need(dlogits, (B, MLP_OUT), torch.float32, "dlogits")
    _need(grad, (MLP_PARAMS,), torch.float32, "grad")
    _check(lib().llp_mlp_backward(B, _ptr(params), _ptr(x), _ptr(act), _ptr(dlogits), _ptr(grad), _stream()))


def mlp_adam(grad, params, m1, m2, step, lr):
    torch = _torch()
    for t, name in ((grad, "grad"), (params, "params"), (m1, "m1"), (m2, "m2")):
        _need(t, (MLP_PARAMS,), torch.float32, name)
    _check(lib().llp_mlp_adam(_ptr(grad), _ptr(params), _ptr(m1), _ptr(m2), int(step), ctypes.c_float(lr),
                              _stream()))


def trace_features(trace, rounds, n, m, kind=KIND_SSSP):
    """features[rounds,12] fp32 (device) of a trace buffer filled by LLP_TRACE
    in a solve of the given kind (KIND_SSSP, KIND_BFS or KIND_JOBS)."""
    torch = _torch()
    if not (isinstance(trace, torch.Tensor) and trace.is_cuda and trace.dtype == torch.uint8
            and trace.is_contiguous() and trace.numel() >= rounds * ctypes.sizeof(TraceRec)):
        raise LLPError(E_ARG, f"trace must be a contiguous uint8 CUDA buffer of at least {rounds} records")
    F = torch.empty((max(rounds, 1), MLP_IN), dtype=torch.float32, device="cuda")
    _check(lib().llp_trace_features(int(rounds), _ptr(trace), int(n), int(m), int(kind), _ptr(F), _stream()))
    return F[:rounds]


def trace_buffer(cap):
    torch = _torch()
    return torch.zeros(cap * ctypes.sizeof(TraceRec), dtype=torch.uint8, device="cuda")


def trace_records(trace, rounds):
    return np.frombuffer(trace.cpu().numpy().tobytes(), TRACE_DTYPE)[:rounds].copy()
