"""GPU parity of the transitive-closure and reduction sweeps against the CPU
oracle (bit-exact), including ragged and degenerate sizes."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")


def tc_case(g):
    csr = llpgen.CSRGraph(g, weighted=False)
    got = llp.transitive_closure(g.n, csr.out_ptr, csr.out_dst)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint32)
    want = oracle.transitive_closure(g.n, g.src, g.dst)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,m,seed", [(1, 0, 1), (5, 3, 2), (33, 40, 3), (100, 60, 4), (1000, 1500, 5)])
def test_tc_uniform(n, m, seed):
    g = llpgen.uniform_graph(n, m, seed=seed, cycle=False) if n > 1 else \
        llpgen.EdgeList(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    tc_case(g)


@pytest.mark.parametrize("n,m,seed", [(4097, 8000, 6), (8192, 65536, 7)])
def test_tc_large_sampled_rows(n, m, seed):
    """At sizes where the literal predicate oracle (cubic per pass) takes minutes,
    sampled rows are checked against breadth-first reachability (paths of
    length >= 1: u itself only when an in-neighbour of u is reachable)."""
    sp = pytest.importorskip("scipy.sparse")
    csg = pytest.importorskip("scipy.sparse.csgraph")
    g = llpgen.uniform_graph(n, m, seed=seed, cycle=False)
    csr = llpgen.CSRGraph(g, weighted=False)
    got = llp.transitive_closure(n, csr.out_ptr, csr.out_dst)
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint32)
    A = sp.csr_matrix((np.ones(g.m, np.int8), (g.src, g.dst)), shape=(n, n))
    words = (n + 31) // 32
    for u in llpgen.uniform_ints(64, 0, n - 1, seed=seed, tag=0x55):
        u = int(u)
        reach = np.zeros(n, bool)
        reach[csg.breadth_first_order(A, u, directed=True, return_predecessors=False)] = True
        ins = g.src[g.dst == u]
        reach[u] = bool(reach[ins].any()) if ins.size else False
        want = np.zeros(words * 32, bool)
        want[:n] = reach
        want_words = np.packbits(want.reshape(-1, 32)[:, ::-1], axis=1).view(">u4").ravel()
        assert np.array_equal(got[u], want_words.astype(np.uint32)), u


def test_tc_self_loop_cycle_and_chain():
    # 0 -> 0 (self-loop), chain 1 -> 2 -> 3, cycle 4 -> 5 -> 4, isolated 6
    src = np.array([0, 1, 2, 4, 5], np.int32)
    dst = np.array([0, 2, 3, 5, 4], np.int32)
    g = llpgen.EdgeList(7, src, dst, np.ones(5, np.int32))
    tc_case(g)
    # a long chain: closure depth n - 1
    n = 3000
    g = llpgen.EdgeList(n, np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32),
                        np.ones(n - 1, np.int32))
    tc_case(g)


def test_tc_rejects_bad_ids():
    ptr = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 7], np.int32)
    with pytest.raises(llp.LLPError) as e:
        llp.transitive_closure(2, ptr, dst)
    assert e.value.status == llp.E_INPUT


@pytest.mark.parametrize("n", [0, 1, 255, 256, 513, 100003, 1 << 24])
def test_reduce(n):
    x = llpgen.u64_words(n, seed=7 + n % 5)
    assert llp.reduce_sum(x) == oracle.reduce_sum(x)


def test_reduce_wraps_and_repeats():
    x = np.full(1000, 2**64 - 1, np.uint64)
    want = oracle.reduce_sum(x)
    assert want == (1000 * (2**64 - 1)) % 2**64
    ws = llp.workspace(llp.KIND_REDUCE, 1000, 0)
    for _ in range(3):                       # the workspace counter resets itself
        assert llp.reduce_sum(x, ws=ws) == want
