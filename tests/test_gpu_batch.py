"""GPU parity of the workgroup-local sweeps: the 0-1 knapsack (single
instance, every launch shape), and the batched persistent solve of mixed
knapsack and small-SSSP instances (plain launch, hipGraph replays, autotuned
shapes) against the CPU oracle, bit-exact per instance."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")

I32 = 2**31 - 1


def want_of(item):
    if item[0] == "knapsack":
        _, wt, val, W = item
        return oracle.knapsack(wt, val, W)
    _, g, s = item
    return oracle.sssp(g.n, g.src, g.dst, g.w, s, bag=True)


def check_batch(items, b):
    got = b.results()
    st = b.status.cpu().numpy()[: len(items)]
    assert (st == 0).all(), np.nonzero(st)[0][:10]
    for i, it in enumerate(items):
        want = want_of(it)
        if it[0] == "knapsack":
            assert got[i] == want, (i, got[i], want)
        else:
            assert np.array_equal(got[i], want), i


# ---------------------------------------------------------------- knapsack
@pytest.mark.parametrize("block", [0, 256, 512, 1024])
@pytest.mark.parametrize("inst", [0, 1, 2, 3])
def test_knapsack_family(inst, block):
    wt, val, W = llpgen.knapsack(inst, seed=5)
    want_best, want_row = oracle.knapsack(wt, val, W, row=True)
    if block == 256 and W + 1 > 256 * 32:
        pytest.skip("W too large for 256 threads")
    best, row = llp.knapsack(wt, val, W, row=True, block=block)
    assert best == want_best
    assert np.array_equal(row.cpu().numpy(), want_row)


def test_knapsack_edge_cases():
    z = np.zeros(0, np.int32)
    assert llp.knapsack(z, z, 0) == 0
    assert llp.knapsack(z, z, 100) == 0
    # W = 0: only weightless items count
    wt = np.array([0, 1, 0], np.int32)
    val = np.array([5, 7, 3], np.int32)
    assert llp.knapsack(wt, val, 0) == oracle.knapsack(wt, val, 0) == 8
    # items heavier than W, zero values, one exact fit
    wt = np.array([11, 10, 3, 7], np.int32)
    val = np.array([100, 9, 0, 4], np.int32)
    assert llp.knapsack(wt, val, 10) == oracle.knapsack(wt, val, 10) == 9
    # largest capacity, ragged item count
    wt = llpgen.uniform_ints(77, 1, 4000, seed=3).astype(np.int32)
    val = llpgen.uniform_ints(77, 1, 1000, seed=4).astype(np.int32)
    wb, wr = oracle.knapsack(wt, val, 16383, row=True)
    b, r = llp.knapsack(wt, val, 16383, row=True)
    assert b == wb and np.array_equal(r.cpu().numpy(), wr)


def test_knapsack_errors():
    wt = np.array([1, 2], np.int32)
    with pytest.raises(llp.LLPError) as e:
        llp.knapsack(wt, np.array([2**30, 2**30 + 5], np.int32), 5)
    assert e.value.status == llp.E_OVERFLOW
    assert oracle.knapsack(wt, np.array([2**30, 2**30 + 5], np.int32), 5, check=False)[0] == llp.E_OVERFLOW
    with pytest.raises(llp.LLPError) as e:
        llp.knapsack(np.array([1, -2], np.int32), np.array([3, 4], np.int32), 5)
    assert e.value.status == llp.E_INPUT
    with pytest.raises(llp.LLPError) as e:
        llp.knapsack(wt, wt, 16384)
    assert e.value.status == llp.E_ARG


# ---------------------------------------------------------------- batch
def small_batch(seed=9, nk=48, ns=48, nhi=700):
    return llpgen.batch_workload(nk, ns, seed=seed, sssp_nhi=nhi)


@pytest.mark.parametrize("shape", [dict(), dict(block=256, chunk=1), dict(block=512, chunk=3),
                                   dict(block=1024, chunk=8)], ids=str)
def test_batch_small_mixed(shape):
    items = small_batch()
    b = llp.Batch(items).solve(**shape)
    torch.cuda.synchronize()
    check_batch(items, b)


def test_batch_edge_instances():
    g1 = llpgen.EdgeList(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    g3 = llpgen.EdgeList(3, np.array([0], np.int32), np.array([1], np.int32), np.array([4], np.int32))
    z = np.zeros(0, np.int32)
    items = [("knapsack", z, z, 0), ("sssp", g1, 0), ("knapsack", np.array([3], np.int32),
                                                     np.array([9], np.int32), 3),
             ("sssp", g3, 0), ("sssp", g3, 2)]
    b = llp.Batch(items).solve()
    torch.cuda.synchronize()
    got = b.results()
    assert got[0] == 0 and got[1].tolist() == [0] and got[2] == 9
    assert got[3].tolist() == [0, 4, I32] and got[4].tolist() == [I32, I32, 0]


def test_batch_largest_instances():
    """The largest instances a batch takes: an SSSP graph of n = 8192 (state,
    two frontier bitmaps and row offsets in LDS) and a knapsack of W = 16383,
    mixed with small ones; the launch's LDS (with the batch kernel's own
    static words) fits one workgroup, and the results equal the oracle's.  One
    vertex more is refused with LLP_E_ARG before anything is launched."""
    rng = np.random.default_rng(12)
    g = llpgen.uniform_graph(8192, 8 * 8192, 1, 100, seed=12)
    wt = rng.integers(1, 4096, size=40).astype(np.int32)
    val = rng.integers(1, 1000, size=40).astype(np.int32)
    items = [("sssp", g, 0), ("knapsack", wt, val, 16383)] + small_batch(seed=12, nk=3, ns=3)
    b = llp.Batch(items).solve()
    torch.cuda.synchronize()
    check_batch(items, b)
    big = llpgen.uniform_graph(8193, 8 * 8193, 1, 100, seed=13)
    with pytest.raises(llp.LLPError) as e:
        llp.Batch([("sssp", big, 0)]).solve()
    assert e.value.status == llp.E_ARG


def test_batch_tuned_block_too_small_for_widest_row(tmp_path):
    """A tuned record is keyed by the instance count only: a record of 256
    threads (at most 8192 knapsack cells per workgroup) for this batch's size
    class must not make a batch with W = 16383 fail; the plan takes 512
    threads instead, and the results equal the oracle's."""
    import json
    rng = np.random.default_rng(14)
    wt = rng.integers(1, 4096, size=24).astype(np.int32)
    val = rng.integers(1, 1000, size=24).astype(np.int32)
    items = [("knapsack", wt, val, 16383)] + small_batch(seed=14, nk=3, ns=4)
    probe = llp.Batch(small_batch(seed=15, nk=4, ns=4))   # the same count, small rows
    assert probe.count == len(items)
    probe.autotune()
    path = tmp_path / "cache.json"
    llp.autotune_save(str(path))
    doc = json.loads(path.read_text())
    cls = len(items).bit_length() - 1
    ents = [e for e in doc["entries"] if e["kind"] == "batch" and e["size_class"] == cls]
    assert ents, doc
    for e in ents:
        e["block"], e["chunk"] = 256, 1
    path.write_text(json.dumps({"llp_autotune": 1, "entries": ents}))
    llp.autotune_load(str(path))
    try:
        assert llp.autotune_lookup(llp.KIND_BATCH, len(items)) == (256, 1)
        b = llp.Batch(items).solve()
        torch.cuda.synchronize()
        check_batch(items, b)
    finally:
        for e in ents:
            e["block"], e["chunk"] = 512, 1
        path.write_text(json.dumps({"llp_autotune": 1, "entries": ents}))
        llp.autotune_load(str(path))


def test_batch_rejects_out_of_range_instance():
    items = small_batch(seed=3, nk=4, ns=4)
    b = llp.Batch(items)
    # shrink the declared pool so the last instance's range falls outside it
    b.pool_words = b.pool_words - 1
    with pytest.raises(llp.LLPError) as e:
        b.solve()
    assert e.value.status == llp.E_INPUT
    st = b.status.cpu().numpy()
    assert (st != 0).sum() >= 1


def test_batch_graph_replays():
    items = small_batch(seed=4)
    b = llp.Batch(items)
    ref = llp.Batch(items).solve()
    torch.cuda.synchronize()
    want = ref.out.cpu().numpy()
    for k in range(4):
        b.out.fill_(-1)                      # eager work between replays
        b.solve(graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(b.out.cpu().numpy(), want), k
    check_batch(items, b)
    # asynchronous replay with a device status word
    sd = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    b.out.fill_(-1)
    b.solve(graph=True, flags=llp.ASYNC, status_dev=sd)
    torch.cuda.synchronize()
    assert int(sd.item()) == 0 and np.array_equal(b.out.cpu().numpy(), want)


def test_batch_autotune():
    items = small_batch(seed=6, nk=64, ns=64)
    b = llp.Batch(items)
    rows = b.autotune()
    assert len(rows) >= 8 and all(ms > 0 for _, _, ms in rows)
    blk, ch = llp.autotune_get()
    assert (blk, ch) in [(r[0], r[1]) for r in rows]
    assert min(rows, key=lambda r: r[2])[:2] == (blk, ch)
    b.out.fill_(-1)
    b.solve()                                 # uses the tuned shape
    torch.cuda.synchronize()
    check_batch(items, b)


def test_batch_full_size():
    """4096 knapsack instances (items U[16,256], W U[256,4096]) mixed with 4096
    SSSP graphs (n U[256,4096], 8n uniform arcs + cycle, w U[1,100]), seed 5,
    one persistent launch, replayed from a hipGraph; every instance checked."""
    items = llpgen.batch_workload(4096, 4096, seed=5)
    b = llp.Batch(items)
    b.solve(graph=True)
    b.out.fill_(-1)
    b.solve(graph=True)
    torch.cuda.synchronize()
    check_batch(items, b)


def test_batch_graph_replay_with_shared_workspace_and_grown_instance():
    """Replays with the library-owned workspace (NULL in opts), which an SSSP
    solve in between overwrites, still solve every instance; after the
    instance table at the same address is edited to hold a larger knapsack
    capacity than the captured launch was sized for, the next replay
    captures again and the result matches the oracle."""
    import ctypes
    items = small_batch(seed=12, nk=24, ns=24)
    b = llp.Batch(items)

    def replay():
        o = llp.make_opts()                      # workspace NULL: the library-owned buffer
        llp._check(llp.lib().llp_solve_batch_graph(*b._args(), ctypes.byref(o)))
        torch.cuda.synchronize()

    replay()
    check_batch(items, b)
    g = llpgen.uniform_graph(4096, 32768, 1, 100, seed=1)
    dg = llp.DeviceGraph(llpgen.CSRGraph(g, weighted=True, out_weights=True))
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gs = dg.cstruct()
    llp._check(llp.lib().llp_solve_sssp(ctypes.byref(gs), 0, llp._ptr(out), ctypes.byref(llp.make_opts())))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.sssp(g.n, g.src, g.dst, g.w, 0))
    b.out.fill_(-1)
    b.status.fill_(-1)
    replay()
    check_batch(items, b)
    # grow one knapsack instance's capacity in place (same arrays, same addresses)
    desc = np.frombuffer(b.desc.cpu().numpy().tobytes(), llp.INSTANCE_DTYPE).copy()
    k = int(np.nonzero(desc["kind"] == llp.KIND_KNAPSACK)[0][0])
    newW = int(desc["cap_or_source"][desc["kind"] == llp.KIND_KNAPSACK].max()) + 3000
    assert newW <= 16383
    desc["cap_or_source"][k] = newW
    b.desc.copy_(torch.from_numpy(desc.view(np.uint8).copy()))
    _, wt, val, _ = items[k]
    items[k] = ("knapsack", wt, val, newW)
    b.out.fill_(-1)
    b.status.fill_(-1)
    replay()
    check_batch(items, b)
