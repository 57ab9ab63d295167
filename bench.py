#!/usr/bin/env python3
"""Benchmark of the LLP sweep on one MI355X.

Workload: R-MAT scale 22 (4,194,304 vertices, 67,108,864 R-MAT arcs with
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), seeded vertex relabelling, plus the
Hamiltonian cycle 0 -> 1 -> ... -> n-1 -> 0: m = 71,303,168 arcs), int32
weights U[1, 255] for SSSP and unit weights for BFS, source = the vertex of
highest out-degree (smallest id on ties).  Synthetic, seeded (seed 22).

One step = one SSSP solve + one BFS solve to the LLP fixpoint on that graph,
inputs resident in HBM.  value = 2 m / step time (GTEPS, every input arc
counted once per solve).  The JSON line also carries each solve's GTEPS, the
roofline of the evaluation kernel (the dominant kernel: pull evaluation of the
candidate worklist), measured with HIP events around each of its launches on
the solve's stream, and the CPU oracle timed on the host on one SSSP solve of
the same graph.
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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--scale", type=int, default=22)
    p.add_argument("--sched", default="plain", choices=["plain", "hybrid", "dense", "push", "learned"])
    p.add_argument("--delta", type=int, default=0,
                   help="delta-bucket width for the fixed schedules (plain becomes fixed pull)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--profile-steps", type=int, default=0,
                   help="run only this many steps, no baseline (for rocprofv3 runs)")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    import llpgen
    import paper_2603_13147_amd as llp

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    t0 = time.time()
    g = llpgen.rmat_graph(a.scale, seed=22)
    src = llpgen.max_outdeg_source(g)
    csr = llpgen.CSRGraph(g, weighted=True, out_weights=True)
    dg = llp.DeviceGraph(csr)
    n, m = g.n, g.m
    print(f"# graph scale {a.scale}: n={n} m={m} source={src} built in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    sched = {"plain": dict(sched=llp.SCHED_PLAIN), "hybrid": dict(sched=llp.SCHED_HYBRID),
             "dense": dict(sched=llp.SCHED_FIXED, flags=llp.DENSE),
             "push": dict(sched=llp.SCHED_FIXED, flags=llp.PUSH),
             "learned": dict(sched=llp.SCHED_LEARNED)}[a.sched]
    if a.delta > 0:
        if sched["sched"] == llp.SCHED_PLAIN:
            sched = dict(sched=llp.SCHED_FIXED)
        sched["delta"] = a.delta
    if a.sched == "learned":
        wpath = os.path.join(ROOT, "paper_2603_13147_amd", "sched_weights.npy")
        llp.set_sched_weights(np.load(wpath))
    ws = llp.workspace(llp.KIND_SSSP, n, m)
    dist = torch.empty(n, dtype=torch.int32, device="cuda")
    lev = torch.empty(n, dtype=torch.int32, device="cuda")

    def step(timing):
        s1, s2 = llp.Stats(), llp.Stats()
        fl = sched.get("flags", 0) | (llp.TIMING if timing else 0)
        kw = dict(sched)
        kw["flags"] = fl
        llp.sssp(dg, src, out=dist, ws=ws, stats=s1, **kw)
        llp.bfs(dg, src, out=lev, ws=ws, stats=s2, **kw)
        return s1, s2

    steps = a.profile_steps or a.steps
    warm = 0 if a.profile_steps else a.warmup
    for _ in range(warm):
        step(False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = [step(True) for _ in range(steps)]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    step_s = (t2 - t1) / steps
    value = 2 * m / step_s / 1e9

    # per-solve rates and the evaluation kernel's roofline (algorithmic bytes:
    # 12 B per SSSP in-arc read (source id, weight, gathered state), 8 B per BFS
    # in-arc (no weight), 16 B per candidate (worklist entry)).
    sssp_ms = np.mean([s1.device_ms for s1, _ in recs])
    bfs_ms = np.mean([s2.device_ms for _, s2 in recs])
    kb = 0.0
    kt = 0.0
    launches = 0
    for s1, s2 in recs:
        kb += 12.0 * s1.edges_inspected + 16.0 * s1.candidates
        kb += 8.0 * s2.edges_inspected + 16.0 * s2.candidates
        kt += s1.kernel_ms + s2.kernel_ms
        launches += s1.eval_launches + s2.eval_launches
    achieved = kb / (kt * 1e-3) / 1e9 if kt > 0 else 0.0
    s1, s2 = recs[-1]
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
                               f"+hamiltonian cycle, w U[1,255] / unit, source max-outdeg",
                   "n": n, "m": m, "schedule": a.sched + (f"+delta{a.delta}" if a.delta else "")},
        "sssp": {"gteps": round(m / (sssp_ms * 1e-3) / 1e9, 4), "ms": round(float(sssp_ms), 3),
                 "rounds": s1.rounds, "edges_inspected": s1.edges_inspected,
                 "expand_edges": s1.expand_edges, "candidates": s1.candidates},
        "bfs": {"gteps": round(m / (bfs_ms * 1e-3) / 1e9, 4), "ms": round(float(bfs_ms), 3),
                "rounds": s2.rounds, "edges_inspected": s2.edges_inspected,
                "expand_edges": s2.expand_edges, "candidates": s2.candidates},
        "roofline": {"kernel": "k_graph_main (pull evaluation)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launches": launches, "avg_launch_us": round(kt * 1e3 / max(launches, 1), 2),
                     "bytes_per_launch": round(kb / max(launches, 1), 1)},
    }
    if not a.no_cpu_baseline and not a.profile_steps:
        import oracle
        t3 = time.perf_counter()
        oracle.sssp(n, g.src, g.dst, g.w, src, bag=True)
        ct = time.perf_counter() - t3
        out["cpu_baseline"] = {"value": round(m / ct / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                               "sample": "one SSSP solve of the same graph by the single-threaded FIFO-bag "
                                         f"oracle ({ct:.1f} s); BFS not timed"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
