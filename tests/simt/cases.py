"""Runs graph-sweep cases on the CPU emulation (tests/simt/_build/
libllp_simt.so) and prints one JSON line per case: the status, the message
and whether the output equals the oracle's.  Started by
tests/test_simt_graph.py in a child process (so a fault or a sanitizer
report ends only that process).  Usage: cases.py <case set>."""
import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
import llpgen  # noqa: E402
import oracle  # noqa: E402
import paper_2603_13147_amd as P  # noqa: E402

L = ctypes.CDLL(os.path.join(HERE, "_build", "libllp_simt.so"))
L.simt_alloc.restype = ctypes.c_void_p
L.simt_alloc.argtypes = [ctypes.c_size_t]
L.simt_free.argtypes = [ctypes.c_void_p]
L.llp_last_error.restype = ctypes.c_char_p
L.llp_workspace_bytes.restype = ctypes.c_size_t
L.llp_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
for fn in (L.llp_solve_sssp, L.llp_solve_bfs):
    fn.argtypes = [ctypes.POINTER(P.Graph), ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(P.Opts)]
L.llp_solve_jobs.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 6 + [ctypes.POINTER(P.Opts)]

SCHEDS = [dict(sched=P.SCHED_PLAIN), dict(sched=P.SCHED_FIXED, flags=P.DENSE),
          dict(sched=P.SCHED_FIXED, flags=P.PUSH), dict(sched=P.SCHED_HYBRID),
          dict(sched=P.SCHED_RANDOM, seed=1), dict(sched=P.SCHED_RANDOM, seed=7),
          dict(sched=P.SCHED_FIXED, delta=40), dict(sched=P.SCHED_FIXED, flags=P.PUSH, delta=7)]


def dev(a):
    """An emulated device copy of a; None (a null pointer, as torch gives) when empty."""
    a = np.ascontiguousarray(a, np.int32)
    if a.nbytes == 0:
        return None
    p = L.simt_alloc(a.nbytes)
    ctypes.memmove(p, a.ctypes.data, a.nbytes)
    return p


def graph(e):
    c = llpgen.CSRGraph(e, weighted=True, out_weights=True)
    g = P.Graph()
    g.n, g.m = c.n, c.m
    g.in_ptr, g.in_src, g.in_w = dev(c.in_ptr), dev(c.in_src), dev(c.in_w)
    g.out_ptr, g.out_dst, g.out_w = dev(c.out_ptr), dev(c.out_dst), dev(c.out_w)
    return g


def solve(kind, g, s, **kw):
    """One solve with a fresh workspace of exactly llp_workspace_bytes, as the binding allocates."""
    o = P.Opts()
    o.size = ctypes.sizeof(P.Opts)
    for k, v in kw.items():
        setattr(o, k, v)
    nb = max(int(L.llp_workspace_bytes(P.KIND_SSSP if kind == "sssp" else P.KIND_BFS, g.n, g.m, None)), 256)
    o.workspace = L.simt_alloc(nb)
    o.workspace_bytes = nb
    outp = L.simt_alloc(4 * g.n)
    fn = L.llp_solve_sssp if kind == "sssp" else L.llp_solve_bfs
    st = fn(ctypes.byref(g), s, outp, ctypes.byref(o))
    out = np.frombuffer((ctypes.c_char * (4 * g.n)).from_address(outp), np.int32).copy()
    msg = L.llp_last_error().decode()
    L.simt_free(o.workspace)
    L.simt_free(outp)
    return st, msg, out


def report(name, e, s, kind, kw, want, stats=False):
    extra = {}
    if stats:
        stt = P.Stats()
        kw = dict(kw)
        kw["flags"] = kw.get("flags", 0) | P.TIMING
        st, msg, got = solve(kind, graph(e), s, stats=ctypes.pointer(stt), **kw)
        extra = {"rounds": int(stt.rounds), "pre_launches": int(stt.pre_launches),
                 "eval_launches": int(stt.eval_launches)}
    else:
        st, msg, got = solve(kind, graph(e), s, **kw)
    print(json.dumps({"case": name, "kind": kind, "source": s, "opts": kw, "status": st, "msg": msg,
                      "equal": bool(np.array_equal(got, want)), **extra}), flush=True)


def edge_cases(sources=range(5), scheds=SCHEDS, isolated=True):
    """n = 1 without arcs; a 5-vertex graph with self-loops, duplicate arcs,
    zero weights, a vertex without out-arcs and an unreachable vertex, from
    every source under every schedule; isolated vertices beside a chain."""
    z = np.zeros(0, np.int32)
    e1 = llpgen.EdgeList(1, z, z, z)
    for kind in ("sssp", "bfs"):
        report("n1", e1, 0, kind, {}, np.zeros(1, np.int32))
    src = np.array([1, 1, 2, 2, 3, 0, 0], np.int32)
    dst = np.array([1, 2, 3, 3, 3, 1, 1], np.int32)
    w = np.array([0, 5, 1, 0, 4, 7, 2], np.int32)
    e5 = llpgen.EdgeList(5, src, dst, w)
    for s in sources:
        ws, wb = oracle.sssp(5, src, dst, w, s), oracle.bfs(5, src, dst, s)
        for kw in scheds:
            report("five", e5, s, "sssp", kw, ws)
            report("five", e5, s, "bfs", kw, wb)
    if not isolated:
        return
    # vertices 0..2 a chain with zero weights, 3..7 isolated, 8 -> 9
    src = np.array([0, 1, 8], np.int32)
    dst = np.array([1, 2, 9], np.int32)
    w = np.array([0, 0, 3], np.int32)
    eiso = llpgen.EdgeList(10, src, dst, w)
    for s in (0, 5, 8):
        for kw in SCHEDS[:4]:
            report("isolated", eiso, s, "sssp", kw, oracle.sssp(10, src, dst, w, s))
            report("isolated", eiso, s, "bfs", kw, oracle.bfs(10, src, dst, s))


def tight_segments():
    """A small graph at the full grid (512 workgroups): each workgroup's list
    segment holds about 200 entries, and bucketed push rounds (random codes,
    fixed buckets) advance far more vertices through the local queues than a
    workgroup's share of the list; every append must still fit."""
    e = llpgen.uniform_graph(1024, 8192, 1, 100, seed=2)
    want = oracle.sssp(e.n, e.src, e.dst, e.w, 0)
    for kw in (dict(sched=P.SCHED_RANDOM, seed=1), dict(sched=P.SCHED_FIXED, flags=P.PUSH, delta=40)):
        report("tight", e, 0, "sssp", kw, want)


def decode_race():
    """4096 vertices (eight 512-vertex decode shares): the launch that finds
    the end decodes G in every workgroup; run in index order, workgroup 0
    first, every later workgroup of that launch must still decode its share."""
    e = llpgen.uniform_graph(4096, 32768, 1, 100, seed=1)
    want = oracle.sssp(e.n, e.src, e.dst, e.w, 0)
    for kw in (dict(sched=P.SCHED_FIXED, flags=P.DENSE), dict(sched=P.SCHED_FIXED, flags=P.PUSH)):
        report("decode", e, 0, "sssp", kw, want)


def tail_cases():
    """Sweeps long enough for the multi-round tail kernel (after the first
    batch of step launches): a 48 x 48 grid (wide buckets under the hybrid,
    none under fixed push, explicit ones), a bare weighted cycle (chains),
    and an R-MAT graph (narrow rounds after dense ones)."""
    e = llpgen.grid_graph(48, 48, 1, 1000, seed=7)
    s = llpgen.max_outdeg_source(e)
    ws, wb = oracle.sssp(e.n, e.src, e.dst, e.w, s, bag=True), oracle.bfs(e.n, e.src, e.dst, s, bag=True)
    for kw in (dict(sched=P.SCHED_HYBRID), dict(sched=P.SCHED_FIXED, flags=P.PUSH),
               dict(sched=P.SCHED_FIXED, flags=P.PUSH, delta=300)):
        report("tail-grid", e, s, "sssp", kw, ws, stats=True)
    report("tail-grid", e, s, "bfs", dict(sched=P.SCHED_HYBRID), wb, stats=True)
    c = llpgen.uniform_graph(2000, 0, 1, 100, seed=31)
    report("tail-chain", c, 0, "sssp", dict(sched=P.SCHED_HYBRID), oracle.sssp(c.n, c.src, c.dst, c.w, 0), stats=True)
    report("tail-chain", c, 0, "bfs", dict(sched=P.SCHED_FIXED, flags=P.PUSH), oracle.bfs(c.n, c.src, c.dst, 0),
           stats=True)
    r = llpgen.rmat_graph(11, seed=5)
    s = llpgen.max_outdeg_source(r)
    report("tail-rmat", r, s, "sssp", dict(sched=P.SCHED_HYBRID), oracle.sssp(r.n, r.src, r.dst, r.w, s, bag=True),
           stats=True)
    report("tail-rmat", r, s, "bfs", dict(sched=P.SCHED_HYBRID), oracle.bfs(r.n, r.src, r.dst, s, bag=True),
           stats=True)


def solve_jobs(pred_ptr, pred_idx, dur, **kw):
    """One readiness sweep (LLP_JOBS_PULL off) on emulated device copies."""
    n = int(dur.shape[0])
    succ_ptr, succ_idx = llpgen.job_succ(pred_ptr, pred_idx)
    o = P.Opts()
    o.size = ctypes.sizeof(P.Opts)
    stt = P.Stats()
    o.stats = ctypes.pointer(stt)
    for k, v in kw.items():
        setattr(o, k, v)
    bufs = [dev(x) for x in (pred_ptr, pred_idx, dur, succ_ptr, succ_idx)]
    outp = L.simt_alloc(4 * n)
    st = L.llp_solve_jobs(n, *bufs, outp, ctypes.byref(o))
    out = np.frombuffer((ctypes.c_char * (4 * n)).from_address(outp), np.int32).copy()
    msg = L.llp_last_error().decode()
    for b in bufs + [outp]:
        if b:
            L.simt_free(b)
    return st, msg, out, int(stt.rounds)


def report_jobs(name, pred_ptr, pred_idx, dur, **kw):
    want_st, want = 0, None
    try:
        want = oracle.jobs(pred_ptr, pred_idx, dur, bag=True)
    except Exception as e:  # a cycle or an overflow: the oracle raises
        want_st = str(e)
    st, msg, got, rounds = solve_jobs(pred_ptr, pred_idx, dur, **kw)
    print(json.dumps({"case": name, "kind": "jobs", "opts": kw, "status": st, "msg": msg,
                      "equal": bool(want is not None and np.array_equal(got, want)), "oracle_error": want_st,
                      "rounds": rounds}), flush=True)


def chain_dag(n, dur=1):
    pred_ptr = np.concatenate([[0], np.arange(n, dtype=np.int32)]).astype(np.int32)
    return pred_ptr, np.arange(n - 1, dtype=np.int32), np.full(n, dur, np.int32)


def diamond_dag(head=50, width=10000, tail=50):
    """A chain of head jobs, the last with width successors, all of which
    precede one job, then a chain of tail jobs: narrow levels, two levels of
    width arcs, narrow levels again."""
    preds = [[]] + [[j - 1] for j in range(1, head)]
    preds += [[head - 1]] * width
    preds += [list(range(head, head + width))]
    preds += [[head + width + i] for i in range(tail)]
    pp = np.concatenate([[0], np.cumsum([len(p) for p in preds])]).astype(np.int32)
    pi = np.array([x for p in preds for x in p], np.int32)
    d = llpgen.uniform_ints(len(preds), 1, 100, seed=12).astype(np.int32)
    return pp, pi, d


def job_cases():
    """The readiness sweep: one job; a 300-job chain (300 levels, one job
    each, most list segments empty); a random DAG; a chain under a round
    limit it passes; a cycle behind a chain; a completion time beyond int32;
    narrow, wide and narrow levels in turn.  Each with the narrow levels run
    by one workgroup (the default), and with one launch per level (suffix
    -l, chunk -1)."""
    pp, pi, d = llpgen.job_dag(3000, 4.0, 1, 1000, seed=9)
    cyc = chain_dag(40)
    cyc[0][0:3] = np.array([0, 1, 2], np.int32)
    cyc = (cyc[0], np.concatenate([[2], cyc[1][1:]]).astype(np.int32), cyc[2])
    for suf, kw in (("", {}), ("-l", dict(chunk=-1))):
        report_jobs("one" + suf, np.array([0, 0], np.int32), np.zeros(0, np.int32), np.array([5], np.int32), **kw)
        report_jobs("chain" + suf, *chain_dag(300, 3), **kw)
        report_jobs("dag" + suf, pp, pi, d, **kw)
        report_jobs("limit" + suf, *chain_dag(100), max_rounds=50, **kw)
        report_jobs("cycle" + suf, *cyc, **kw)
        report_jobs("overflow" + suf, *chain_dag(20, 1 << 28), **kw)
        report_jobs("diamond" + suf, *diamond_dag(), **kw)


if __name__ == "__main__":
    {"edge": edge_cases,
     "edge-wide": lambda: (edge_cases(sources=(0, 2), scheds=SCHEDS[:4], isolated=False), tight_segments()),
     "decode": decode_race, "tail": tail_cases, "jobs": job_cases}[sys.argv[1]]()
