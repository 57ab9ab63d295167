"""GPU parity of the stable-marriage and job-scheduling sweeps against the CPU
oracle (bit-exact int32) for every schedule, at small, ragged and full sizes,
plus warm starts and error paths.  Calls go through the C ABI."""
import numpy as np
import pytest

import llpgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
llp = pytest.importorskip("paper_2603_13147_amd")

I32 = 2**31 - 1

SM_SCHEDS = [
    dict(),                                             # unbounded chains, one launch
    dict(chunk=1),                                      # one proposal per thread per round
    dict(chunk=5),
    dict(sched=llp.SCHED_FIXED, flags=llp.DENSE),       # dense rounds
    dict(sched=llp.SCHED_RANDOM, seed=3),               # dense rounds, seeded coin flips
]


def sm_ids(k):
    return "-".join(f"{a}{b}" for a, b in k.items()) or "chains"


def run_sm(mpref, wrank, **kw):
    wife, prop = llp.stable_marriage(mpref, wrank, **kw)
    torch.cuda.synchronize()
    return wife.cpu().numpy(), prop.cpu().numpy()


@pytest.mark.parametrize("kw", SM_SCHEDS, ids=sm_ids)
@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (7, 3), (64, 4), (300, 5)])
def test_sm_small_all_schedules(n, seed, kw):
    mpref, wrank = llpgen.sm_prefs(n, seed=seed)
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    w, p = run_sm(mpref, wrank, **kw)
    assert np.array_equal(w, want_w)
    assert np.array_equal(p, want_p)


@pytest.mark.parametrize("kw", SM_SCHEDS[:3], ids=sm_ids)
def test_sm_full_size_8192(kw):
    """n = 8192 men and women, uniform random full lists (seed 3)."""
    mpref, wrank = llpgen.sm_prefs(8192, seed=3)
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    w, p = run_sm(mpref, wrank, **kw)
    assert np.array_equal(w, want_w)
    assert np.array_equal(p, want_p)


@pytest.mark.parametrize("kw", [dict(), dict(chunk=4)], ids=["lds", "grid"])
def test_sm_largest_lds_instance(kw):
    """n = 12288, the largest instance the single-workgroup path takes
    (default schedule), and the grid-wide chains on the same lists."""
    mpref, wrank = llpgen.sm_prefs(12288, seed=8)
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    w, p = run_sm(mpref, wrank, **kw)
    assert np.array_equal(w, want_w)
    assert np.array_equal(p, want_p)


def test_sm_same_list_worst_case():
    # every man has the same list and every woman the same ranking: the
    # proposal count is n (n + 1) / 2, the deepest displacement chains; men
    # reach list positions up to n - 1, past the 64 the (woman, rank) table holds
    n = 200
    mpref = np.tile(np.arange(n, dtype=np.int16), (n, 1))
    wrank = np.tile(np.arange(n, dtype=np.int16), (n, 1))
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    for kw in SM_SCHEDS:
        w, p = run_sm(mpref, wrank, **kw)
        assert np.array_equal(w, want_w) and np.array_equal(p, want_p), kw


def test_sm_warm_start_and_stats():
    mpref, wrank = llpgen.sm_prefs(1000, seed=11)
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    st = llp.Stats()
    w, p = run_sm(mpref, wrank, stats=st, flags=llp.TIMING)
    assert np.array_equal(p, want_p)
    assert st.advances >= 1000 and st.rounds == 1 and st.device_ms > 0
    # warm start from a state below the fixpoint (half of every index)
    warm = torch.from_numpy((want_p // 2).astype(np.int32)).cuda()
    w2, p2 = run_sm(mpref, wrank, warm_start=warm)
    assert np.array_equal(p2, want_p) and np.array_equal(w2, want_w)


def test_sm_validation():
    mpref, wrank = llpgen.sm_prefs(50, seed=2)
    bad = mpref.copy()
    bad[7, 3] = bad[7, 4]            # not a permutation
    with pytest.raises(llp.LLPError) as e:
        run_sm(bad, wrank, flags=llp.VALIDATE)
    assert e.value.status == llp.E_INPUT
    badr = wrank.copy()
    badr[3, 0] = 50                  # rank out of range
    with pytest.raises(llp.LLPError) as e:
        run_sm(mpref, badr, flags=llp.VALIDATE)
    assert e.value.status == llp.E_INPUT
    # valid input passes validation
    want_w, _ = oracle.stable_marriage(mpref, wrank)
    w, _ = run_sm(mpref, wrank, flags=llp.VALIDATE)
    assert np.array_equal(w, want_w)


def test_sm_not_converged():
    mpref, wrank = llpgen.sm_prefs(300, seed=9)
    with pytest.raises(llp.LLPError) as e:
        run_sm(mpref, wrank, chunk=1, max_rounds=2)
    assert e.value.status == llp.E_NOT_CONVERGED


# ---------------------------------------------------------------- jobs
JOB_SCHEDS = [
    dict(),                                                        # readiness counters
    dict(chunk=-1),                                                # the same, one launch per level
    dict(pull=True),                                               # pull, worklists
    dict(pull=True, sched=llp.SCHED_FIXED, flags=llp.DENSE),
    dict(pull=True, sched=llp.SCHED_FIXED, flags=llp.PUSH),
    dict(pull=True, sched=llp.SCHED_HYBRID),
    dict(pull=True, sched=llp.SCHED_RANDOM, seed=5),
]


def job_ids(k):
    return "-".join(f"{a}{b}" for a, b in k.items()) or "ready"


def run_jobs(pp, pi, d, **kw):
    sp, si = llpgen.job_succ(pp, pi)
    out = llp.jobs(pp, pi, d, sp, si, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kw", JOB_SCHEDS, ids=job_ids)
@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (10, 3), (1000, 4), (65537, 6)])
def test_jobs_all_schedules(n, seed, kw):
    pp, pi, d = llpgen.job_dag(n, seed=seed)
    want = oracle.jobs(pp, pi, d, bag=n > 2000)
    assert np.array_equal(run_jobs(pp, pi, d, **kw), want)


@pytest.mark.parametrize("kw", JOB_SCHEDS[:4], ids=job_ids)
def test_jobs_full_size(kw):
    """2^20 jobs, in-degree min(Poisson(8), j) over lower ids, durations U[1,1000] (seed 4)."""
    pp, pi, d = llpgen.job_dag(1 << 20, seed=4)
    want = oracle.jobs(pp, pi, d, bag=True)
    st = llp.Stats()
    got = run_jobs(pp, pi, d, stats=st, **kw)
    assert np.array_equal(got, want)
    if not kw.get("pull"):
        # every job with successors is listed once when fixed; every arc is read once
        sp, _ = llpgen.job_succ(pp, pi)
        assert st.advances == int((np.diff(sp) > 0).sum()) and st.edges_inspected == pi.shape[0]


def test_jobs_chain_and_isolated():
    # a 3000-job chain (depth 3000) and jobs without arcs
    n = 3000
    pp = np.concatenate([[0, 0], np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    pi = np.arange(0, n - 1, dtype=np.int32)
    d = llpgen.uniform_ints(n, 0, 1000, seed=8).astype(np.int32)
    want = oracle.jobs(pp, pi, d)
    for kw in JOB_SCHEDS[:3]:
        assert np.array_equal(run_jobs(pp, pi, d, **kw), want), kw
    z = np.zeros(5, np.int32)
    assert run_jobs(np.zeros(6, np.int32), np.zeros(0, np.int32), z + 3).tolist() == [0] * 5


@pytest.mark.parametrize("kw", JOB_SCHEDS[:2], ids=job_ids)
def test_jobs_long_chain_and_round_limit(kw):
    # 9000 levels, one job each: launch batches up to their largest size, most
    # list segments empty; by default 64 levels per launch in one workgroup
    n = 9000
    pp = np.concatenate([[0, 0], np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    pi = np.arange(0, n - 1, dtype=np.int32)
    d = llpgen.uniform_ints(n, 0, 100, seed=9).astype(np.int32)
    want = oracle.jobs(pp, pi, d)
    st = llp.Stats()
    assert np.array_equal(run_jobs(pp, pi, d, stats=st, **kw), want)
    assert st.rounds == n - 1
    # a round limit below the depth ends the sweep with LLP_E_NOT_CONVERGED
    st = llp.Stats()
    with pytest.raises(llp.LLPError) as e:
        run_jobs(pp, pi, d, max_rounds=100, stats=st, **kw)
    assert e.value.status == llp.E_NOT_CONVERGED


def test_jobs_history_batches_on_reused_arrays():
    """The first batch of level launches is sized from the last sweep of the
    same arrays: a 3000-level chain and a two-level star with the same array
    shapes, written in turn into the same device tensors, each solved against
    the oracle (a stale history only changes how many launches are enqueued)."""
    n = 3000
    pp = np.concatenate([[0, 0], np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    chain = np.arange(0, n - 1, dtype=np.int32)
    star = np.zeros(n - 1, np.int32)
    d = llpgen.uniform_ints(n, 0, 1000, seed=10).astype(np.int32)
    dev = [torch.from_numpy(x).cuda() for x in (pp, chain, d) + llpgen.job_succ(pp, chain)]
    for pi in (chain, chain, star, chain, star):
        sp, si = llpgen.job_succ(pp, pi)
        dev[1].copy_(torch.from_numpy(pi))
        dev[3].copy_(torch.from_numpy(sp))
        dev[4].copy_(torch.from_numpy(si))
        st = llp.Stats()
        got = llp.jobs(*dev, stats=st)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), oracle.jobs(pp, pi, d))
        assert st.rounds == (n - 1 if pi is chain else 1)


def cyclic_jobs():
    # 0 -> 1 -> 2 -> 0 plus 3 <- 2
    preds = {0: [2], 1: [0], 2: [1], 3: [2]}
    pp = np.zeros(5, np.int32)
    pi = []
    for j in range(4):
        pi += preds[j]
        pp[j + 1] = len(pi)
    return pp, np.array(pi, np.int32), np.array([1, 2, 3, 4], np.int32)


def test_jobs_cycle():
    pp, pi, d = cyclic_jobs()
    with pytest.raises(oracle.OracleError):
        oracle.jobs(pp, pi, d)
    for kw in (dict(), dict(pull=True)):
        with pytest.raises(llp.LLPError) as e:
            run_jobs(pp, pi, d, **kw)
        assert e.value.status == llp.E_CYCLE, kw


def test_jobs_overflow_and_validation():
    n = 4
    pp = np.array([0, 0, 1, 2, 3], np.int32)
    pi = np.array([0, 1, 2], np.int32)
    d = np.array([2**30, 2**30, 2**30, 5], np.int32)
    assert oracle.jobs(pp, pi, d, check=False)[0] == llp.E_OVERFLOW
    for kw in (dict(), dict(pull=True)):
        with pytest.raises(llp.LLPError) as e:
            run_jobs(pp, pi, d, **kw)
        assert e.value.status == llp.E_OVERFLOW, kw
    # successor lists that do not match the predecessor lists
    pp, pi, d = llpgen.job_dag(100, seed=2)
    sp, si = llpgen.job_succ(pp, pi)
    si = si.copy()
    si[5] = (si[5] + 1) % 100
    with pytest.raises(llp.LLPError) as e:
        llp.jobs(pp, pi, d, sp, si, flags=llp.VALIDATE)
    assert e.value.status == llp.E_INPUT


def test_jobs_repeated_solves_equal_the_oracle():
    """30 readiness solves of one 2^18-job DAG (wide levels and runs of narrow
    ones) in each form: narrow levels in one workgroup up to 1024 arcs, up to
    256 arcs (more hand-overs between the forms), and one launch per level.
    Every output equals the oracle's, whatever order the workgroups run in."""
    pp, pi, d = llpgen.job_dag(1 << 18, seed=21)
    sp, si = llpgen.job_succ(pp, pi)
    want = oracle.jobs(pp, pi, d)
    dev = [torch.from_numpy(x).cuda() for x in (pp, pi, d, sp, si)]
    for i in range(30):
        for kw in (dict(), dict(chunk=256), dict(chunk=-1)):
            st = llp.Stats()
            got = llp.jobs(*dev, stats=st, **kw)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (i, kw)
            assert st.rounds > 1


def test_sm_repeated_solves_equal_the_oracle():
    """20 solves of one n = 4096 instance in the single-workgroup chain form
    and in the grid chain form, on device tensors reused across runs: the
    chains interleave differently from run to run, but the man-optimal
    matching is unique, and every run returns the oracle's."""
    mpref, wrank = llpgen.sm_prefs(4096, seed=22)
    want_w, want_p = oracle.stable_marriage(mpref, wrank)
    mp, wr = torch.from_numpy(mpref).cuda(), torch.from_numpy(wrank).cuda()
    for i in range(20):
        for kw in (dict(), dict(chunk=4)):
            w, p = run_sm(mp, wr, **kw)
            assert np.array_equal(w, want_w), (i, kw)
            assert np.array_equal(p, want_p), (i, kw)
