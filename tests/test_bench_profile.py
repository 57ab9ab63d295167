"""Host logic of the bench's per-phase profile summary (no GPU): the step
launches of each traced solve map to rounds in order, a push round to one PRE
launch, a dense round to one MAIN launch, a pull round and a BFS bitmap dense
round to PRE then MAIN; launches past the last round and after a tail launch
are not mapped.  And the algorithmic bytes of a solve, with and without
bitmap rounds."""
import csv
import importlib.util
import json
import os
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def write_trace(d, names, log):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for i, n in enumerate(names):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Start_Timestamp": t, "End_Timestamp": t + 1000 * (i + 1)})
            t += 100000
    with open(os.path.join(d, "round_log.json"), "w") as f:
        json.dump(log, f)


INIT = "llp::k_graph_init(llp::GArgs, int const*)"
STEP = "void llp::k_graph_step<false, true>(llp::GArgs, int)"
TAIL = "llp::k_graph_tail(llp::GArgs, int)"
PUSH, DENSE, PULL = 2, 1, 0


def test_phases_with_bitmap_rounds(tmp_path):
    b = load_bench()
    # an untraced warm-up solve, then two logged solves:
    #   bfs: push, bitmap dense, plain dense, push, then one no-op launch
    #   sssp: pull, push, then a tail launch and a step launch after it
    names = [INIT, STEP, STEP,
             INIT] + [STEP] * 6 + [INIT] + [STEP] * 3 + [TAIL, STEP]
    log = [{"solve": "bfs", "modes": [PUSH, DENSE, DENSE, PUSH], "bitmap": [0, 1, 0, 0]},
           {"solve": "sssp", "modes": [PULL, PUSH], "bitmap": [0, 0]}]
    write_trace(str(tmp_path), names, log)
    ph = b.step_phases(str(tmp_path))
    ids = {k: [r[0] for r in v] for k, v in ph.items()}
    # solve 1 dispatches 5..10: push 5 (pre), bitmap round 6 (pre) + 7 (main),
    # dense 8 (main), push 9 (pre), no-op 10 left out
    # solve 2 dispatches 12..16: pull 12 (pre) + 13 (main), push 14 (pre), tail 15, after it 16
    assert ids["pre"] == [5, 6, 9, 12, 14]
    assert ids["main"] == [7, 8, 13]
    assert ids["tail"] == [15]
    assert ids["after_tail"] == [16]


def test_kernel_bytes_prices_the_bitmap():
    b = load_bench()
    s = types.SimpleNamespace(edges_inspected=100, states_gathered=40, candidates=10, advances=7,
                              expand_edges=5, push_edges=3, bitmap_rounds=0)
    n = 1024
    main, pre = b.kernel_bytes(s, True, n)
    assert main == 8 * 100 + 4 * 40 + 16 * 10
    assert pre == 16 * 7 + 8 * 5 + 12 * 3
    s.bitmap_rounds = 2
    main2, pre2 = b.kernel_bytes(s, False, n)
    # unit weights: 4 B per arc, the bitmap read once per round by MAIN; PRE
    # reads the n states and writes the bitmap once per round
    assert main2 == 4 * 100 + 4 * 40 + 16 * 10 + 2 * (n // 8)
    assert pre2 == 16 * 7 + 8 * 5 + 8 * 3 + 2 * 4 * n + 2 * (n // 8)


def test_cli_refuses_several_gpus_and_needs_one():
    """--gpus above 1 exits with a message (the sweep does not shard); without
    a visible GPU the bench prints an error line instead of a measurement."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert json.loads(r.stdout.strip().splitlines()[-1])["n_gpus"] == 2
    import torch
    if not torch.cuda.is_available():
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup", "0"],
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 1
        assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_committed_traffic_follows_the_kernel_sources(tmp_path):
    """The bench reports the committed counter traffic of a phase only while
    the step kernel's sources hash as they did when the counters were taken:
    the committed summary matches the tree as it is, and a one-byte change to
    a kernel source (in a copy of the tree) turns the figure into None."""
    import shutil
    b = load_bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_graph_step_rmat22_hybrid.traffic.json")))
    assert b.committed_traffic("main") == rec["phases"]["main"]["traffic_bytes_per_launch"]
    assert b.committed_traffic("pre") == rec["phases"]["pre"]["traffic_bytes_per_launch"]
    assert b.committed_traffic("tail") is None
    csrc = tmp_path / "paper_2603_13147_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in b.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2603_13147_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "k_graph_step_rmat22_hybrid.traffic.json"), tmp_path / "profiles")
    b.ROOT = str(tmp_path)
    assert b.committed_traffic("main") == rec["phases"]["main"]["traffic_bytes_per_launch"]
    with open(csrc / b.KERNEL_SOURCES[0], "ab") as f:
        f.write(b"\n")
    assert b.committed_traffic("main") is None
