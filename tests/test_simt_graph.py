"""The graph sweep's kernels on the CPU emulation of tests/simt: cases kept
off the GPU (degenerate graphs) and a regression test of the launch that
decodes the output, checked against the oracle.  The kernels and host code
are the product's own sources compiled with g++ (AddressSanitizer when
available) against tests/simt/hip/hip_runtime.h; every guard that fires
surfaces as a nonzero status."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "simt"))
import build as simt_build  # noqa: E402


@pytest.fixture(scope="module")
def simt_lib():
    return simt_build.build()


def run_cases(which, cus, timeout=900):
    env = dict(os.environ)
    asan = simt_build.asan_runtime()
    if asan:
        env["LD_PRELOAD"] = asan
        env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0"
    env["SIMT_CUS"] = str(cus)
    r = subprocess.run([sys.executable, os.path.join(HERE, "simt", "cases.py"), which], env=env,
                       capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, r.stderr[-4000:]
    return [json.loads(line) for line in r.stdout.splitlines() if line.startswith("{")]


def test_degenerate_graphs(simt_lib):
    """n = 1 without arcs, zero weights, self-loops, duplicate arcs, a source
    without out-arcs, unreachable and isolated vertices; SSSP and BFS from
    every source under every schedule, 4 workgroups per launch."""
    rows = run_cases("edge", 2)
    assert len(rows) == 2 + 5 * 8 * 2 + 3 * 4 * 2
    bad = [r for r in rows if r["status"] != 0 or not r["equal"]]
    assert not bad, bad[:5]


def test_degenerate_graphs_full_grid(simt_lib):
    """The same graphs with 512 workgroups per launch, as on the MI355X (far
    more list segments and waves than arcs): n = 1, and the 5-vertex graph
    from a source with duplicate arcs and from one with zero-weight arcs
    under the plain, dense, push and hybrid schedules; and bucketed push
    rounds whose local queues advance more vertices than a workgroup's list
    segment was sized for."""
    rows = run_cases("edge-wide", 256)
    assert len(rows) == 2 + 2 * 4 * 2 + 2
    bad = [r for r in rows if r["status"] != 0 or not r["equal"]]
    assert not bad, bad[:5]


def test_decode_by_every_workgroup(simt_lib):
    rows = run_cases("decode", 8)
    assert len(rows) == 2
    assert all(r["status"] == 0 and r["equal"] for r in rows), rows


def test_tail_rounds_and_local_queues(simt_lib):
    """The multi-round tail kernel (a cooperative launch whose workgroups run
    consecutive push rounds between barriers, here 4 of them interleaved by
    the emulation) takes over once a sweep outlasts the first batch of step
    launches with narrow push rounds; bucketed push rounds drain their
    bucket through each workgroup's local queue.  On a grid (hybrid with wide
    buckets, fixed push, explicit buckets, BFS) and a bare cycle every
    output equals the oracle's; the unbucketed long sweeps run most rounds in
    one tail launch, and the hybrid's bucketed sweep of the grid needs only
    a few rounds."""
    rows = run_cases("tail", 16)
    assert len(rows) == 8
    assert all(r["status"] == 0 and r["equal"] for r in rows), [r for r in rows if not r["equal"]]
    long = [r for r in rows if r["case"] in ("tail-grid", "tail-chain") and "delta" not in r["opts"]
            and not (r["case"] == "tail-grid" and r["kind"] == "sssp" and r["opts"]["sched"] == 3)]
    assert len(long) == 4
    assert all(r["pre_launches"] <= 17 and r["rounds"] > 40 for r in long), long
    hyb = [r for r in rows if r["case"] == "tail-grid" and r["kind"] == "sssp" and r["opts"]["sched"] == 3][0]
    assert hyb["rounds"] <= 8, hyb
    dlt = [r for r in rows if "delta" in r["opts"]][0]
    assert dlt["rounds"] <= 100, dlt


def test_jobs_levels(simt_lib):
    """The readiness sweep, with its narrow levels run by one workgroup in
    LDS and with one launch per level (suffix -l): one job, a 300-level
    chain, a random DAG, a round limit it runs past, a cycle, a completion
    time beyond int32, and narrow levels around two of 10000 arcs; statuses,
    rounds and start times against the oracle."""
    by = {r["case"]: r for r in run_cases("jobs", 16)}
    names = {"one", "chain", "dag", "limit", "cycle", "overflow", "diamond"}
    assert set(by) == names | {x + "-l" for x in names}
    for suf in ("", "-l"):
        for name in ("one", "chain", "dag", "diamond"):
            assert by[name + suf]["status"] == 0 and by[name + suf]["equal"], by[name + suf]
        assert by["chain" + suf]["rounds"] == 299 and by["one" + suf]["rounds"] == 0
        assert by["diamond" + suf]["rounds"] == 101
        assert by["dag" + suf]["rounds"] == by["dag"]["rounds"]
        assert by["limit" + suf]["status"] == 5 and by["limit" + suf]["rounds"] == 50       # LLP_E_NOT_CONVERGED
        assert by["cycle" + suf]["status"] == 8 and by["cycle" + suf]["oracle_error"]        # LLP_E_CYCLE
        assert by["overflow" + suf]["status"] == 4 and by["overflow" + suf]["oracle_error"]  # LLP_E_OVERFLOW
