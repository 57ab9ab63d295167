#!/usr/bin/env python3
"""Benchmark of the LLP sweep on one MI355X.

Headline workload: R-MAT scale 22 (4,194,304 vertices, 67,108,864 R-MAT arcs
with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), seeded vertex relabelling, plus
the Hamiltonian cycle 0 -> 1 -> ... -> n-1 -> 0: m = 71,303,168 arcs), int32
weights U[1, 255] for SSSP and unit weights for BFS, source = the vertex of
highest out-degree (smallest id on ties).  Synthetic, seeded (seed 22).

One step = one SSSP solve + one BFS solve to the LLP fixpoint on that graph,
inputs resident in HBM, with the headline schedule (the frontier-width
hybrid: dense rounds when the changed vertices' out-arcs exceed a third of
the arcs for SSSP and 1/14 for BFS, push rounds otherwise).  value = 2 m / step
time (GTEPS, every input arc counted once per solve).

The JSON line also carries
  - each solve's GTEPS, rounds and work counters;
  - the learned-vs-plain comparison on the same graph (and the other fixed
    schedules), plus the held-out evaluation graphs of the learned scheduler
    (R-MAT 22 seed 900, 4096^2 grid seed 900) when --heldout is given;
  - the batched persistent solve: 4096 knapsack + 4096 small SSSP instances
    in one hipGraph-replayed launch (solves/s, median of 21 replays), the
    same instances solved one by one through the single-instance entry
    points (the batched-vs-plain speedup), per-kind rates and floors;
  - the roofline of the dominant kernel of the headline step (the kernel with
    the most device time: PRE = expansion / push, MAIN = pull evaluation),
    from HIP events around each of its launches on the solve's stream;
  - the CPU oracle timed on the host on one full step of the same graph (an
    SSSP and a BFS solve, adjacency lists built before the clock starts),
    with binary-heap Dijkstra and queue BFS beside it, the host CPU model
    and the CPUs visible.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
# sources of the step kernel, hashed to tell whether committed counters still apply
KERNEL_SOURCES = ("graph.hip", "llp_lists.h", "llp_sched.h", "llp_dev.h")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--sched", default="auto", choices=["auto", "plain", "hybrid", "dense", "push", "learned"])
    p.add_argument("--delta", type=int, default=0,
                   help="delta-bucket width for the fixed schedules (plain becomes fixed pull)")
    p.add_argument("--wgs-per-cu", type=int, default=0, help="graph sweep workgroups per CU (0 = default)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-compare", action="store_true", help="skip the schedule comparison")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-solve measurement")
    p.add_argument("--heldout", action="store_true", help="also time the learned scheduler's held-out graphs")
    p.add_argument("--profile-steps", type=int, default=0,
                   help="run only this many headline steps, nothing else (for rocprofv3 runs)")
    p.add_argument("--round-log", default="",
                   help="with --profile-steps: write the round codes of the event-timed solves to this JSON file "
                        "(maps a kernel trace's step launches to phases: one per push round, two per pull or "
                        "dense round)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only copy a 1 GiB device buffer 3 times (reference for rocprofv3 byte counters)")
    p.add_argument("--calibrate-gather", action="store_true",
                   help="only gather 2^25 4-byte values at random and in order from a 16 MB and a 4 GiB "
                        "table, twice each (what rocprofv3 byte counters read per random gather)")
    p.add_argument("--summarize-profile", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                   help="summarise rocprofv3 output directories of --profile-steps runs (each holding the "
                        "round log written with --round-log as round_log.json) and of --calibrate-copy runs: "
                        "per-phase launches, durations and byte counters of the step kernel; writes the "
                        "traffic record the bench reads and prints a Markdown table (no GPU needed)")
    return p.parse_args()


BATCH_REPLAYS = 21
LDS_PEAK_BS = 128 * 256 * 2.4e9   # MI355X LDS: 128 B per clock per CU, 256 CUs, 2.4 GHz


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batch_replay_ms(llp, b, torch):
    """Median device time of BATCH_REPLAYS hipGraph replays (after the capture)."""
    b.solve(graph=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(BATCH_REPLAYS):
        st = llp.Stats()
        b.solve(graph=True, stats=st, flags=llp.TIMING)
        ts.append(st.device_ms)
    return float(np.median(ts))


def one_by_one(llp, items, b, res, torch):
    """The batch's instances solved one at a time through the single-instance
    entry points (llp_solve_knapsack, llp_solve_sssp: synchronous calls, inputs
    already on the device, one workspace sized for the largest instance), with
    the plain schedule and with the hybrid one; wall time of the whole loop and
    equality of every output with the batch's."""
    import ctypes
    import llpgen
    L = llp.lib()
    prep = []
    nmax = mmax = 1
    for it in items:
        if it[0] == "knapsack":
            _, wt, val, W = it
            prep.append(("k", llp._dev(wt, torch.int32), llp._dev(val, torch.int32), int(W)))
        else:
            _, g, s = it
            dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
            prep.append(("s", dg, dg.cstruct(), int(s)))
            nmax, mmax = max(nmax, g.n), max(mmax, int(g.m))
    ws = llp.workspace(llp.KIND_SSSP, nmax, mmax)
    best = torch.zeros(len(items), dtype=torch.int32, device="cuda")
    dist = torch.zeros(max(int(b.out_words), 1), dtype=torch.int32, device="cuda")
    got = {}
    for name, sched in (("plain", llp.SCHED_PLAIN), ("hybrid", llp.SCHED_HYBRID)):
        o = llp.make_opts(workspace=ws, sched=sched)
        ok = llp.make_opts(workspace=ws)
        ptrs = []
        for i, p in enumerate(prep):
            a, k = b.out_slices[i]
            if p[0] == "k":
                ptrs.append((0, p, best.data_ptr() + 4 * i))
            else:
                ptrs.append((1, p, dist.data_ptr() + 4 * a))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for kind, p, optr in ptrs:
            if kind == 0:
                st = L.llp_solve_knapsack(len(p[1]), p[3], llp._ptr(p[1]), llp._ptr(p[2]), ctypes.c_void_p(optr),
                                          None, ctypes.byref(ok))
            else:
                st = L.llp_solve_sssp(ctypes.byref(p[2]), p[3], ctypes.c_void_p(optr), ctypes.byref(o))
            if st:
                raise llp.LLPError(st, L.llp_last_error().decode())
        torch.cuda.synchronize()
        got[name] = (time.perf_counter() - t0) * 1e3
    # equality with the batch: knapsack bests and SSSP distances
    r = res.cpu().numpy()
    bb, dd = best.cpu().numpy(), dist.cpu().numpy()
    equal = True
    for i, p in enumerate(prep):
        a, k = b.out_slices[i]
        if p[0] == "k":
            equal &= int(bb[i]) == int(r[a])
        else:
            equal &= bool(np.array_equal(dd[a:a + k], r[a:a + k]))
    return {"plain_ms": round(got["plain"], 1), "hybrid_ms": round(got["hybrid"], 1),
            "bit_exact_vs_batch": bool(equal),
            "how": "each instance by its own synchronous llp_solve_knapsack / llp_solve_sssp call (inputs on the "
                   "device, outputs written in place), wall time of the loop"}


def sched_kw(llp, name, delta=0):
    kw = {"plain": dict(sched=llp.SCHED_PLAIN), "hybrid": dict(sched=llp.SCHED_HYBRID),
          "dense": dict(sched=llp.SCHED_FIXED, flags=llp.DENSE),
          "push": dict(sched=llp.SCHED_FIXED, flags=llp.PUSH),
          "learned": dict(sched=llp.SCHED_LEARNED)}[name]
    if delta > 0:
        if kw["sched"] == llp.SCHED_PLAIN:
            kw = dict(sched=llp.SCHED_FIXED)
        kw["delta"] = delta
    return kw


def run_step(llp, dg, src, ws, dist, lev, kw, timing, log=None):
    """One headline step (SSSP then BFS).  log: a list that receives the
    round codes of both solves (traced with LLP_TRACE)."""
    s1, s2 = llp.Stats(), llp.Stats()
    k = dict(kw)
    k["flags"] = k.get("flags", 0) | (llp.TIMING if timing else 0)
    if log is None:
        llp.sssp(dg, src, out=dist, ws=ws, stats=s1, **k)
        llp.bfs(dg, src, out=lev, ws=ws, stats=s2, **k)
        return s1, s2
    k["flags"] |= llp.TRACE
    for name, fn, out, st in (("sssp", llp.sssp, dist, s1), ("bfs", llp.bfs, lev, s2)):
        trace = llp.trace_buffer(8192)
        fn(dg, src, out=out, ws=ws, stats=st, trace=trace, **k)
        rec = llp.trace_records(trace, int(st.rounds))
        log.append({"solve": name, "modes": [int(c) for c in rec["mode"]],
                    "bitmap": [int(b) for b in rec["bitmap"]]})
    return s1, s2


def kernel_bytes(s, weighted, n):
    """Algorithmic bytes of the MAIN (pull evaluation) and PRE (expansion / push)
    kernels of one solve: MAIN reads per in-arc the source id and the weight
    (SSSP; 8 / 4 B), per gathered tail state 4 B (a dense round does not
    gather the arcs that cannot improve their row) and 16 B per candidate
    entry, and a BFS bitmap round reads the n-bit bitmap once; PRE reads 16 B
    per changed entry, per expansion arc the target id and its stamp (8 B),
    per push arc the target id, weight and state (12 / 8 B), and for a bitmap
    round the n states (4 B each) and writes the bitmap."""
    arc = 12 if weighted else 8
    bm = s.bitmap_rounds * (n // 8)
    main = (arc - 4) * s.edges_inspected + 4 * s.states_gathered + 16 * s.candidates + bm
    pre = 16 * s.advances + 8 * s.expand_edges + arc * s.push_edges + s.bitmap_rounds * 4 * n + bm
    return main, pre


def committed_traffic(phase):
    """HBM bytes per launch of the given phase of the step kernel from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by a plain
    copy's counters), or None when none was taken for that phase or the kernel
    sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_graph_step_rmat22_hybrid.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2603_13147_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                for f in KERNEL_SOURCES)).hexdigest()[:16]
    ph = rec.get("phases", {}).get(phase)
    return ph["traffic_bytes_per_launch"] if (h == rec["source_sha16"] and ph) else None


def _csv_rows(d, suffix):
    """Rows of the rocprofv3 CSV file ending in suffix under directory d."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def _dispatches(d):
    """(dispatch id, kernel name, duration us or None, {counter: value}) per
    dispatch, in dispatch order, from a kernel trace or a counter collection."""
    import glob
    recs = {}
    if glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in _csv_rows(d, "counter_collection.csv"):
            k = int(r["Dispatch_Id"])
            e = recs.setdefault(k, [k, r["Kernel_Name"], None, {}])
            e[3][r["Counter_Name"]] = e[3].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    else:
        for r in _csv_rows(d, "kernel_trace.csv"):
            k = int(r["Dispatch_Id"])
            recs[k] = [k, r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3, {}]
    return [recs[k] for k in sorted(recs)]


def step_phases(d):
    """Phase of every step-kernel dispatch of the event-timed solves of a
    --profile-steps run: the solves are cut at k_graph_init, the last ones
    paired with the round log, and each solve's step launches before its
    first multi-round (tail) launch mapped to its rounds in order (a push
    round one PRE launch, a dense round one MAIN launch, a pull round and a
    BFS dense round with the bitmap (marked in the trace) PRE then MAIN; launches
    past the last round are no-ops).  Returns {phase: [dispatch]}
    with phases pre, main, tail (the multi-round launches) and after_tail
    (step launches after one, not mapped)."""
    import re
    log = json.load(open(os.path.join(d, "round_log.json")))
    solves, cur = [], None
    for rec in _dispatches(d):
        name = rec[1]
        if "k_graph_init" in name:
            cur = []
            solves.append(cur)
        elif cur is not None and ("k_graph_step" in name or re.search(r"k_graph_tail\b(?!_)", name)):
            cur.append(rec)
    if len(solves) < len(log):
        raise SystemExit(f"{d}: {len(solves)} solves traced, {len(log)} in the round log")
    out = {"pre": [], "main": [], "tail": [], "after_tail": []}
    for launches, ent in zip(solves[-len(log):], log):
        want = []
        for code, bm in zip(ent["modes"], ent["bitmap"]):
            mode = code & 3
            dense = ["pre", "main"] if bm else ["main"]
            want += ["pre", "main"] if mode == 0 else (dense if mode == 1 else ["pre"])
        i = 0
        for j, rec in enumerate(launches):
            if "k_graph_tail" in rec[1]:
                out["tail"].append(rec)
                out["after_tail"] += [x for x in launches[j + 1:] if "k_graph_step" in x[1]]
                out["tail"] += [x for x in launches[j + 1:] if "k_graph_tail" in x[1]]
                break
            if i < len(want):
                out[want[i]].append(rec)
                i += 1
    return out


def summarize_profile(dirs):
    """Per-phase figures of the step kernel from rocprofv3 runs; writes
    profiles/k_graph_step_rmat22_hybrid.traffic.json."""
    import hashlib
    trace, fetch, write, cfetch, cwrite = dirs
    copied = 1 << 30   # --calibrate-copy: 2^28 int32 per copy

    def copy_kib(d, counter):
        v = [r[3][counter] for r in _dispatches(d) if counter in r[3] and "copy" in r[1].lower()]
        v = v or [r[3][counter] for r in _dispatches(d) if counter in r[3]]
        return float(np.median(v))
    fs = copied / (copy_kib(cfetch, "FETCH_SIZE") * 1024)
    ws_ = copied / (copy_kib(cwrite, "WRITE_SIZE") * 1024)
    pt, pf, pw = step_phases(trace), step_phases(fetch), step_phases(write)
    csrc = os.path.join(ROOT, "paper_2603_13147_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                for f in KERNEL_SOURCES)).hexdigest()[:16]
    phases = {}
    print("| phase | launches | trace avg us | FETCH_SIZE KiB / launch | WRITE_SIZE KiB / launch | "
          "HBM traffic / launch |")
    print("|---|---|---|---|---|---|")
    for ph in ("pre", "main", "tail", "after_tail"):
        if not pt[ph]:
            continue
        us = float(np.mean([r[2] for r in pt[ph]]))
        fk = float(np.mean([r[3]["FETCH_SIZE"] for r in pf[ph]])) if pf[ph] else 0.0
        wk = float(np.mean([r[3]["WRITE_SIZE"] for r in pw[ph]])) if pw[ph] else 0.0
        fb, wb = int(fk * 1024 * fs), int(wk * 1024 * ws_)
        phases[ph] = {"launches_traced": len(pt[ph]), "avg_us_trace": round(us, 2),
                      "fetch_kib_per_launch": round(fk, 1), "write_kib_per_launch": round(wk, 1),
                      "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                      "traffic_bytes_per_launch": fb + wb}
        print(f"| {ph.upper()} | {len(pt[ph])} | {us:.2f} | {fk:.0f} | {wk:.0f} | {(fb + wb) / 1e6:.1f} MB |")
    rec = {"kernel": "k_graph_step", "workload": "rmat22 sssp+bfs hybrid", "source_sha16": h,
           "fetch_scale": round(fs, 4), "write_scale": round(ws_, 4), "phases": phases}
    path = os.path.join(ROOT, "profiles", "k_graph_step_rmat22_hybrid.traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"\ncopy scale factors: FETCH_SIZE {fs:.4f}, WRITE_SIZE {ws_:.4f}; sources {h}; wrote {path}")


def calibrate_gather(torch):
    """2^25 random and in-order 4-byte gathers (torch.take, int64 indices)
    from a 16 MB table (the R-MAT 22 state array's size: larger than an XCD's
    L2, within the Infinity Cache) and a 4 GiB one (beyond both); two of each.
    Dispatch order: per table, randint, arange, remainder, then take(random),
    take(in order) twice."""
    n = 1 << 25
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    res = []
    for name, tn in (("16MB", 1 << 22), ("4GiB", 1 << 30)):
        t = torch.ones(tn, dtype=torch.int32, device="cuda")
        ridx = torch.randint(0, tn, (n,), device="cuda", generator=g)
        sidx = torch.arange(n, device="cuda") % tn
        torch.cuda.synchronize()
        for _ in range(2):
            for kind, idx in (("random", ridx), ("in_order", sidx)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                torch.take(t, idx)
                e1.record()
                torch.cuda.synchronize()
                res.append({"table": name, "kind": kind, "ms": round(e0.elapsed_time(e1), 4)})
        del t, ridx, sidx
    print(json.dumps({"gathers_per_launch": n, "index_bytes": 8, "launches": res}), flush=True)


def time_steps(llp, dg, src, ws, dist, lev, kw, steps, warm, torch, log=None):
    """Wall time per step over `steps` steps without per-launch events, then
    the same number of steps with LLP_TIMING for the kernel counters (their
    round codes go to `log` when given)."""
    for _ in range(warm):
        run_step(llp, dg, src, ws, dist, lev, kw, False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        run_step(llp, dg, src, ws, dist, lev, kw, False)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t1) / steps
    recs = [run_step(llp, dg, src, ws, dist, lev, kw, True, log) for _ in range(steps)]
    torch.cuda.synchronize()
    return t, recs


def main():
    a = parse()
    if a.summarize_profile:
        summarize_profile(a.summarize_profile)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the bench runs on one GPU (the sweep does not shard); --gpus above 1 is not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import llpgen
    import paper_2603_13147_amd as llp

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if a.calibrate_gather:
        calibrate_gather(torch)
        return
    if a.calibrate_copy:
        x = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes_per_launch": x.numel() * 4, "launches": 3}), flush=True)
        return
    wpath = llp.default_sched_weights_path()
    have_w = os.path.exists(wpath)
    if have_w:
        llp.set_sched_weights(np.load(wpath))
    # headline: the frontier-width hybrid (dense above m/3 arcs for SSSP, m/14 for BFS),
    # the fastest schedule measured on this graph; the learned and plain
    # schedules are reported beside it
    head = a.sched if a.sched != "auto" else "hybrid"
    if head == "learned" and not have_w:
        print(json.dumps({"error": f"{wpath} is missing: train the scheduler first"}))
        sys.exit(1)

    t0 = time.time()
    g = llpgen.rmat_graph(a.scale, seed=22)
    src = llpgen.max_outdeg_source(g)
    csr = llpgen.CSRGraph(g, weighted=True, out_weights=True)
    dg = llp.DeviceGraph(csr)
    n, m = g.n, g.m
    print(f"# graph scale {a.scale}: n={n} m={m} source={src} built in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ws = llp.workspace(llp.KIND_SSSP, n, m, a.wgs_per_cu)
    dist = torch.empty(n, dtype=torch.int32, device="cuda")
    lev = torch.empty(n, dtype=torch.int32, device="cuda")

    kw = sched_kw(llp, head, a.delta)
    if a.wgs_per_cu:
        kw["chunk"] = a.wgs_per_cu
    steps = a.profile_steps or a.steps
    warm = 0 if a.profile_steps else a.warmup
    log = [] if (a.profile_steps and a.round_log) else None
    step_s, recs = time_steps(llp, dg, src, ws, dist, lev, kw, steps, warm, torch, log)
    if log is not None:
        with open(a.round_log, "w") as f:
            json.dump(log, f)
    value = 2 * m / step_s / 1e9
    print(f"# headline {head}: {step_s * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    # dominant kernel of the headline step and its roofline
    mb = pb = mt = pt = 0.0
    ml = pl = 0
    for s1, s2 in recs:
        for s, weighted in ((s1, True), (s2, False)):
            x, y = kernel_bytes(s, weighted, n)
            mb += x
            pb += y
            mt += s.kernel_ms
            pt += s.pre_ms
            ml += s.eval_launches
            pl += s.pre_launches
    if pt > mt:
        kname, kb, kt, kl = "k_graph_pre (successor expansion / push)", pb, pt, pl
    else:
        kname, kb, kt, kl = "k_graph_main (pull evaluation)", mb, mt, ml
    achieved = kb / (kt * 1e-3) / 1e9 if kt > 0 else 0.0
    traffic = committed_traffic("pre" if pt > mt else "main")
    s1, s2 = recs[-1]
    sssp_ms = float(np.mean([r[0].device_ms for r in recs]))
    bfs_ms = float(np.mean([r[1].device_ms for r in recs]))
    out = {
        "metric": "SSSP/BFS GTEPS to LLP fixpoint",
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"rmat-scale{a.scale} sssp+bfs (a,b,c,d)=(.57,.19,.19,.05), relabelled, "
                               f"+hamiltonian cycle, w U[1,255] / unit, source max-outdeg, seed 22",
                   "n": n, "m": m, "schedule": head + (f"+delta{a.delta}" if a.delta else "")},
        "sssp": {"gteps": round(m / (sssp_ms * 1e-3) / 1e9, 4), "ms": round(sssp_ms, 3),
                 "rounds": s1.rounds, "edges_inspected": s1.edges_inspected,
                 "states_gathered": s1.states_gathered, "push_edges": s1.push_edges,
                 "expand_edges": s1.expand_edges, "candidates": s1.candidates},
        "bfs": {"gteps": round(m / (bfs_ms * 1e-3) / 1e9, 4), "ms": round(bfs_ms, 3),
                "rounds": s2.rounds, "edges_inspected": s2.edges_inspected,
                 "states_gathered": s2.states_gathered, "push_edges": s2.push_edges,
                "expand_edges": s2.expand_edges, "candidates": s2.candidates},
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launches": kl, "avg_launch_us": round(kt * 1e3 / max(kl, 1), 2),
                     "bytes_per_launch": round(kb / max(kl, 1), 1),
                     "other_kernel_ms_per_step": round((mt if pt > mt else pt) / steps, 3)},
    }
    if a.profile_steps:
        print(json.dumps(out), flush=True)
        return

    if not a.no_compare:
        cmp = {}
        for name in ["plain", "hybrid", "push", "dense"] + (["learned"] if have_w else []):
            t, rr = time_steps(llp, dg, src, ws, dist, lev, sched_kw(llp, name), 3, 1, torch)
            cmp[name] = {"ms_per_step": round(t * 1e3, 3),
                         "sssp_ms": round(float(np.mean([r[0].device_ms for r in rr])), 3),
                         "bfs_ms": round(float(np.mean([r[1].device_ms for r in rr])), 3)}
            print(f"# {name}: {t * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
        entry = {"schedules": cmp}
        if have_w:
            entry["speedup_learned_vs_plain"] = round(cmp["plain"]["ms_per_step"] / cmp["learned"]["ms_per_step"], 3)
            entry["speedup_learned_vs_hybrid"] = round(cmp["hybrid"]["ms_per_step"] / cmp["learned"]["ms_per_step"], 3)
        out["learned_vs_plain"] = entry

    if a.heldout and have_w:
        held = {}
        for name, gg in (("rmat22-s900", llpgen.rmat_graph(22, seed=900)),
                         ("grid4096-s900", llpgen.grid_graph(4096, 4096, seed=900))):
            s = llpgen.max_outdeg_source(gg)
            dgh = llp.DeviceGraph(llpgen.CSRGraph(gg, weighted=True, out_weights=True))
            wsh = llp.workspace(llp.KIND_SSSP, gg.n, gg.m)
            o1 = torch.empty(gg.n, dtype=torch.int32, device="cuda")
            o2 = torch.empty(gg.n, dtype=torch.int32, device="cuda")
            res = {}
            for nm, o in (("plain", o1), ("learned", o2)):
                st = llp.Stats()
                llp.sssp(dgh, s, out=o, ws=wsh, **sched_kw(llp, nm))           # warm
                llp.sssp(dgh, s, out=o, ws=wsh, stats=st, flags=llp.TIMING, **sched_kw(llp, nm))
                res[nm] = round(st.device_ms, 3)
            torch.cuda.synchronize()
            held[name] = {"sssp_plain_ms": res["plain"], "sssp_learned_ms": res["learned"],
                          "speedup": round(res["plain"] / res["learned"], 3),
                          "bit_exact": bool(torch.equal(o1, o2))}
            print(f"# held-out {name}: {held[name]}", file=sys.stderr, flush=True)
            del dgh, wsh, o1, o2
        out.setdefault("learned_vs_plain", {})["heldout_sssp"] = held

    if not a.no_batch:
        items = llpgen.batch_workload(4096, 4096, seed=5)
        b = llp.Batch(items)
        tune = b.autotune()                      # launch shape (threads, instances per claim)
        med = batch_replay_ms(llp, b, torch)
        res = b.out.clone()
        # the same instances one kind at a time (their own batches), for per-kind rates
        kn = [it for it in items if it[0] == "knapsack"]
        ss = [it for it in items if it[0] == "sssp"]
        kn_ms = batch_replay_ms(llp, llp.Batch(kn), torch)
        ss_ms = batch_replay_ms(llp, llp.Batch(ss), torch)
        cells = sum(len(it[1]) * (it[3] + 1) for it in kn)
        arcs = sum(int(it[1].m) for it in ss)
        in_bytes = 4 * b.pool_words + b.desc.numel() + 4 * b.out_words
        one = one_by_one(llp, items, b, res, torch)
        out["batch"] = {"workload": "4096 knapsack (items U[16,256], W U[256,4096]) + 4096 sssp "
                                    "(n U[256,4096], 8n arcs + cycle, w U[1,100]), seed 5, hipGraph replay",
                        "instances": b.count, "ms": round(med, 3), "replays": BATCH_REPLAYS,
                        "solves_per_s": round(b.count / (med * 1e-3), 1),
                        "tuned_shape": list(llp.autotune_get()),
                        "untuned_ms": {f"{bl}x{ch}": ms for bl, ch, ms in tune},
                        "knapsack_only_ms": round(kn_ms, 3), "sssp_only_ms": round(ss_ms, 3),
                        "knapsack_cells": cells, "knapsack_gcells_per_s": round(cells / (kn_ms * 1e-3) / 1e9, 2),
                        # a DP cell is one LDS row write and one shifted LDS read (8 B):
                        # LDS peak 128 B per clock per CU x 256 CUs x 2.4 GHz
                        "knapsack_lds_frac": round(8 * cells / (kn_ms * 1e-3) / LDS_PEAK_BS, 4),
                        "sssp_arcs": arcs, "sssp_garcs_per_s": round(arcs / (ss_ms * 1e-3) / 1e9, 2),
                        "hbm_floor_us": round(in_bytes / (HBM_PEAK_GBS * 1e9) * 1e6, 1),
                        "hbm_floor_frac": round(in_bytes / (HBM_PEAK_GBS * 1e9) / (med * 1e-3), 4),
                        "one_by_one": one,
                        "speedup_batched_vs_plain": round(one["plain_ms"] / med, 1),
                        "speedup_batched_vs_hybrid": round(one["hybrid_ms"] / med, 1)}
        print(f"# batch: {med:.3f} ms; one by one: plain {one['plain_ms']:.1f} ms, hybrid {one['hybrid_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    if not a.no_batch:
        # the other plugins at their full sizes (stable marriage n = 8192,
        # seed 3; job DAG of 2^20 jobs, seed 4): median device time of 3 solves
        def med_ms(fn):
            ts = []
            for _ in range(4):
                st = llp.Stats()
                fn(st)
                ts.append(st.device_ms)
            return float(np.median(ts[1:]))
        mp, wr = llpgen.sm_prefs(8192, seed=3)
        mpd, wrd = torch.from_numpy(mp).cuda(), torch.from_numpy(wr).cuda()
        wsm = llp.workspace(llp.KIND_SM, 8192, 0)
        sm_ms = med_ms(lambda st: llp.stable_marriage(mpd, wrd, ws=wsm, stats=st, flags=llp.TIMING))
        st = llp.Stats()
        llp.stable_marriage(mpd, wrd, ws=wsm, stats=st)
        out["stable_marriage"] = {"n": 8192, "ms": round(sm_ms, 3), "solves_per_s": round(1e3 / sm_ms, 1),
                                  "proposals": st.advances,
                                  "advances_per_s": round(st.advances / (sm_ms * 1e-3), 1)}
        del mpd, wrd
        pp, pi, du = llpgen.job_dag(1 << 20, seed=4)
        sp, si = llpgen.job_succ(pp, pi)
        dev = [torch.from_numpy(x).cuda() for x in (pp, pi, du, sp, si)]
        wsj = llp.workspace(llp.KIND_JOBS, 1 << 20, int(pi.shape[0]))
        jr = med_ms(lambda st: llp.jobs(*dev, ws=wsj, stats=st, flags=llp.TIMING))
        # the pull form is the generic sweep: timed with the headline's hybrid
        # schedule and with the plain one
        jp = med_ms(lambda st: llp.jobs(*dev, ws=wsj, stats=st, flags=llp.TIMING, pull=True,
                                        sched=llp.SCHED_HYBRID))
        jpp = med_ms(lambda st: llp.jobs(*dev, ws=wsj, stats=st, flags=llp.TIMING, pull=True))
        st = llp.Stats()
        llp.jobs(*dev, ws=wsj, stats=st)
        # one bulk pass reads per arc the successor id, the parent's start and
        # duration (12 B) and per job its two row offsets and start (12 B)
        bulk = 12 * int(pi.shape[0]) + 12 * (1 << 20)
        out["jobs"] = {"n": 1 << 20, "arcs": int(pi.shape[0]), "readiness_ms": round(jr, 3), "pull_ms": round(jp, 3),
                       "pull_plain_ms": round(jpp, 3), "levels": st.rounds,
                       "us_per_level": round(jr * 1e3 / max(st.rounds, 1), 2),
                       "bulk_pass_floor_us": round(bulk / (HBM_PEAK_GBS * 1e9) * 1e6, 1),
                       "bulk_pass_frac": round(bulk / (HBM_PEAK_GBS * 1e9) / (jr * 1e-3), 4)}
        print(f"# stable marriage {sm_ms:.3f} ms, jobs {jr:.3f} / {jp:.3f} (plain {jpp:.3f}) ms", file=sys.stderr,
              flush=True)

    if not a.no_cpu_baseline:
        import oracle
        # one headline step (an SSSP and a BFS solve) by the single-threaded
        # FIFO-bag oracle, adjacency lists built before its clock starts;
        # binary-heap Dijkstra and queue BFS timed beside it for context
        d_cpu, t_s = oracle.sssp_bag_timed(n, g.src, g.dst, g.w, src)
        l_cpu, t_b = oracle.sssp_bag_timed(n, g.src, g.dst, None, src)
        _, t_dj = oracle.dijkstra_timed(n, g.src, g.dst, g.w, src)
        _, t_q = oracle.bfs_queue_timed(n, g.src, g.dst, src)
        out["cpu_baseline"] = {"value": round(2 * m / (t_s + t_b) / 1e9, 6), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one full step of the same graph (FIFO-bag oracle SSSP {t_s:.1f} s + BFS "
                                         f"{t_b:.1f} s, adjacency built beforehand, 1 thread)",
                               "gpu_output_equal": bool(np.array_equal(d_cpu, dist.cpu().numpy())
                                                        and np.array_equal(l_cpu, lev.cpu().numpy())),
                               "dijkstra_s": round(t_dj, 3), "queue_bfs_s": round(t_q, 3),
                               "host_cpu": host_cpu(), "host_cpus_visible": len(os.sched_getaffinity(0))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
