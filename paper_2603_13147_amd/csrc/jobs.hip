// jobs.hip - earliest start times of a job DAG (paper Section 5.5) on gfx950,
// with the paper's readiness counters.
//
// State.  S[j] is the start time of job j (bottom 0); alpha(S, j) is the
// largest S[p] + dur[p] over its predecessors p.  The paper adds readiness to
// the predicate: a job is only evaluated once every predecessor is fixed, so
// each job is advanced exactly once, to its final value, and the work is
// proportional to the arcs.
//
// Rounds.  Round r consumes the list R[r-1] of jobs that became ready (fixed)
// in round r-1 and walks their successor arcs, edge-balanced across waves:
// each arc (p -> j) publishes S[p] + dur[p] into S[j] with atomicMax and
// decrements j's counter of unfixed predecessors; the arc that brings the
// counter to zero appends j to R[r].  Every contribution to S[j] is made in an
// earlier launch than the one that reads S[j] (j is read only when R[r] is
// consumed by round r+1), so the kernel boundary orders them.  A round with
// an empty input list ends the sweep; a job whose counter never reached zero
// lies on (or after) a cycle.  The pull form of the sweep (LLP_JOBS_PULL)
// runs in the generic graph sweep.
#include <string.h>

#include "llp_host.h"
#include "llp_lists.h"

namespace llp {

constexpr int JB = 256;            // threads per workgroup
constexpr int JW = JB / LLP_WAVE;  // waves per workgroup
constexpr int J_MAX_SEG = 1024;

struct JCtrl {
    int done;
    int status;
    int last_round;
    int pad;
    int diag[8];
    long long rounds, ready, edges;
};

struct JArgs {
    int n, E;
    const int* pred_ptr;
    const int* pred_idx;
    const int* dur;
    const int* succ_ptr;
    const int* succ_idx;
    int* S;
    int* cnt;          // unfixed predecessors per job
    ListRef l0, l1;
    int nseg;
    JCtrl* ctrl;
};

struct JShared {
    int cnt[J_MAX_SEG];
    int epre[J_MAX_SEG + 1];
    int own[JW][64];
    unsigned long long ctr;
    int tot_edges, tot_count;
    int tmp[JW + 1];
};

__device__ __forceinline__ ListRef jl_of(const JArgs& a, int r) { return (r & 1) ? a.l1 : a.l0; }

__global__ void k_jobs_init(JArgs a, const int* warm) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long j = tid; j < a.n; j += nt) {
        int s = warm ? warm[j] : 0;
        a.S[j] = s > 0 ? s : 0;
        a.cnt[j] = a.pred_ptr[j + 1] - a.pred_ptr[j];
    }
    for (long long s = tid; s < a.nseg; s += nt) {
        a.l0.seg[s] = 0ull;
        a.l1.seg[s] = 0ull;
    }
    if (tid == 0) {
        JCtrl c;
        memset(&c, 0, sizeof(c));
        *a.ctrl = c;
    }
}

// Validation: row offsets, ids, durations, and that the successor lists hold
// the same arcs as the predecessor lists (per-job counts; cnt is the
// scratch counter here and is re-initialised afterwards).
__global__ void k_jobs_validate_count(JArgs a) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    for (long long j = tid; j <= a.n; j += nt) {
        int p = a.pred_ptr[j], q = a.succ_ptr[j];
        if (j == 0 && (p != 0 || q != 0)) bad = true;
        if (j == a.n && (p != a.E || q != a.E)) bad = true;
        if (j < a.n) {
            if (a.pred_ptr[j + 1] < p || a.succ_ptr[j + 1] < q) bad = true;
            if (a.dur[j] < 0) bad = true;
        }
    }
    for (long long e = tid; e < a.E; e += nt) {
        int x = a.pred_idx[e], y = a.succ_idx[e];
        if (x < 0 || x >= a.n || y < 0 || y >= a.n) {
            bad = true;
            continue;
        }
        aadd(&a.cnt[y], -1);
    }
    if (bad) set_status(&a.ctrl->status, LLP_E_INPUT);
}

__global__ void k_jobs_validate_check(JArgs a) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long j = tid; j < a.n; j += nt)
        if (a.cnt[j] != 0) set_status(&a.ctrl->status, LLP_E_INPUT);
}

// R[0]: the jobs without predecessors.  Workgroup b seeds a contiguous block
// of jobs into its own segment.
__global__ void __launch_bounds__(JB) k_jobs_seed(JArgs a) {
    __shared__ unsigned long long ctr;
    if (ld_relaxed(&a.ctrl->status)) return;
    if (threadIdx.x == 0) ctr = 0ull;
    __syncthreads();
    const int per = (a.n + gridDim.x - 1) / gridDim.x;
    const int b = blockIdx.x * per, e = min(b + per, a.n);
    for (int base = b; base < e; base += JB) {
        int j = base + threadIdx.x;
        bool ready = false;
        int sb = 0, deg = 0;
        if (j < e) {
            ready = a.pred_ptr[j + 1] == a.pred_ptr[j];
            sb = a.succ_ptr[j];
            deg = a.succ_ptr[j + 1] - sb;
        }
        append(ready && deg > 0, j, sb, deg, &ctr, a.l0, &a.ctrl->status);
    }
    __syncthreads();
    if (threadIdx.x == 0) a.l0.seg[blockIdx.x] = ctr;
}

__device__ __forceinline__ void jobs_wave_range(int total, int& wb, int& we) {
    const long long W = (long long)gridDim.x * JW;
    const long long w = (long long)blockIdx.x * JW + (threadIdx.x >> 6);
    wb = (int)((long long)total * w / W);
    we = (int)((long long)total * (w + 1) / W);
}

__global__ void __launch_bounds__(JB) k_jobs_level(JArgs a, int r) {
    __shared__ JShared sh;
    JCtrl* c = a.ctrl;
    if (ld_relaxed(&c->done) || ld_relaxed(&c->status)) return;
    const ListRef in = jl_of(a, r - 1);
    const ListRef out = jl_of(a, r);
    load_segments(in.seg, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);
    if (sh.tot_count == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->done = 1;
            c->last_round = r - 1;
        }
        return;
    }
    if (threadIdx.x == 0) sh.ctr = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->rounds = r;
        c->ready += sh.tot_count;
        c->edges += sh.tot_edges;
    }
    __syncthreads();
    SegView sv{in.ent, in.cap, a.nseg, sh.cnt, sh.epre, sh.tot_edges, sh.tot_count};
    ListSrc src{sv, c->diag};
    int wb, we;
    jobs_wave_range(sh.tot_edges, wb, we);
    int* own = sh.own[threadIdx.x >> 6];
    bool ovf = false;
    for_edges(src, wb, we, own, [&](const EdgeCtx& x) {
        // completion time of each window entry, handed to its arcs
        long long cm = 0;
        if (x.mine_valid) {
            int p = guard(x.mine.x, a.n, c->diag, 71);
            cm = (long long)a.S[p] + a.dur[p];
        }
        if (cm > LLP_INF) {
            ovf = true;
            cm = LLP_INF;
        }
        int cp = shfl((int)cm, x.j);
        bool ready = false;
        int j = 0, sb = 0, deg = 0;
        if (x.active) {
            int e = guard(x.csr, a.E, c->diag, 72, x.own.x, x.own.y);
            j = guard(a.succ_idx[e], a.n, c->diag, 73, e);
            amax(&a.S[j], cp);
            ready = aadd(&a.cnt[j], -1) == 1;
            if (ready) {
                sb = a.succ_ptr[j];
                deg = a.succ_ptr[j + 1] - sb;
            }
        }
        append(ready && deg > 0, j, sb, deg, &sh.ctr, out, &c->status);
    });
    __syncthreads();
    if (threadIdx.x == 0) out.seg[blockIdx.x] = sh.ctr;
    if (__any(ovf) && lane() == 0) set_status(&c->status, LLP_E_OVERFLOW);
}

// Completion times must fit int32; a job never made ready lies on a cycle.
__global__ void k_jobs_final(JArgs a) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    bool ovf = false, cyc = false;
    for (long long j = tid; j < a.n; j += nt) {
        if ((long long)a.S[j] + a.dur[j] > LLP_INF) ovf = true;
        if (a.cnt[j] != 0) cyc = true;
    }
    if (cyc) set_status(&a.ctrl->status, LLP_E_CYCLE);
    if (ovf) set_status(&a.ctrl->status, LLP_E_OVERFLOW);
}

// --------------------------------------------------------------- host
struct JobsLayout {
    int nseg;
    int cap;
};

static JobsLayout jobs_layout(int64_t n, int64_t E) {
    JobsLayout L;
    // half a segment per CU: levels hold a few thousand jobs and every workgroup
    // first scans all segment counts (at 2^20 jobs, 128 segments beat 256 by 2%; 64 lose 14%)
    L.nseg = device_info().cus / 2;
    if (L.nseg > J_MAX_SEG) L.nseg = J_MAX_SEG;
    if (L.nseg < 1) L.nseg = 1;
    long long W = (long long)L.nseg * JW;
    long long per_wave = (E + W - 1) / W;
    long long cap_level = JW * per_wave + JW * 2 + 64;
    long long cap_seed = (n + L.nseg - 1) / L.nseg + 64;
    L.cap = (int)(cap_level > cap_seed ? cap_level : cap_seed);
    return L;
}

static size_t jobs_ws(int64_t n, int64_t E, JArgs* a, char* base, size_t cap) {
    JobsLayout L = jobs_layout(n, E);
    Carver cv{base, cap, 0, base == nullptr};
    int* cnt = cv.take<int>(n);
    JCtrl* ctrl = cv.take<JCtrl>(1);
    ListRef lists[2];
    for (int i = 0; i < 2; ++i) {
        lists[i].seg = cv.take<unsigned long long>(L.nseg);
        lists[i].ent = cv.take<int4>((size_t)L.nseg * L.cap);
        lists[i].cap = L.cap;
        lists[i].segmin = nullptr;
    }
    if (a) {
        a->cnt = cnt;
        a->ctrl = ctrl;
        a->l0 = lists[0];
        a->l1 = lists[1];
        a->nseg = L.nseg;
    }
    return cv.used;
}

// the pull form shares the graph sweep's workspace
size_t graph_workspace_bytes(int64_t n, int64_t m, int chunk);

size_t jobs_workspace_bytes(int64_t n, int64_t E, int chunk) {
    size_t a = jobs_ws(n, E, nullptr, nullptr, 0);
    size_t b = graph_workspace_bytes(n, E, chunk);
    return a > b ? a : b;
}

int solve_jobs_pull(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx, const int32_t* dur,
                    const int32_t* succ_ptr, const int32_t* succ_idx, int32_t* start, const llp_opts* opts,
                    int64_t E);

static int grid1(int64_t work) {
    int64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    int cap = device_info().cus * 8;
    return (int)(g < cap ? g : cap);
}

int solve_jobs(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx, const int32_t* dur,
               const int32_t* succ_ptr, const int32_t* succ_idx, int32_t* start, const llp_opts* opts) {
    if (n <= 0) return fail(LLP_E_ARG, "n must be positive (got %d)", n);
    if (!pred_ptr || !dur || !succ_ptr || !start)
        return fail(LLP_E_ARG, "pred_ptr, dur, succ_ptr and start are required");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    // the arc count is the last row offset
    int E = 0;
    int s = readback(st, pred_ptr + n, &E, sizeof(int));
    if (s) return s;
    if (E < 0) return fail(LLP_E_INPUT, "pred_ptr[n] is negative");
    if (E > 0 && (!pred_idx || !succ_idx)) return fail(LLP_E_ARG, "pred_idx and succ_idx are required");
    if (o.flags & LLP_JOBS_PULL) return solve_jobs_pull(n, pred_ptr, pred_idx, dur, succ_ptr, succ_idx, start, opts, E);
    if (o.sched != LLP_SCHED_PLAIN)
        return fail(LLP_E_ARG, "the readiness schedule takes no schedule options (use LLP_JOBS_PULL)");

    JArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.E = E;
    a.pred_ptr = pred_ptr;
    a.pred_idx = pred_idx;
    a.dur = dur;
    a.succ_ptr = succ_ptr;
    a.succ_idx = succ_idx;
    a.S = start;
    size_t need = jobs_ws(n, E, nullptr, nullptr, 0);
    void* ws = nullptr;
    s = get_workspace(o, need, &ws);
    if (s) return s;
    jobs_ws(n, E, &a, (char*)ws, need);

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    const int g1 = grid1((int64_t)n > E ? n : E);
    hipLaunchKernelGGL(k_jobs_init, dim3(grid1(n)), dim3(256), 0, st, a, o.warm_start);
    if (o.flags & LLP_VALIDATE) {
        hipLaunchKernelGGL(k_jobs_validate_count, dim3(g1), dim3(256), 0, st, a);
        hipLaunchKernelGGL(k_jobs_validate_check, dim3(grid1(n)), dim3(256), 0, st, a);
        JCtrl h0;
        s = readback(st, a.ctrl, &h0, sizeof(h0));
        if (s) return s;
        if (h0.status) return fail(LLP_E_INPUT, "job lists failed validation (offsets, ids, durations or arc sets)");
        hipLaunchKernelGGL(k_jobs_init, dim3(grid1(n)), dim3(256), 0, st, a, o.warm_start);
    }
    hipLaunchKernelGGL(k_jobs_seed, dim3(a.nseg), dim3(JB), 0, st, a);
    LLP_HIP(hipGetLastError());

    const int64_t max_rounds = o.max_rounds > 0 ? o.max_rounds : (int64_t)n + 2;
    JCtrl h;
    memset(&h, 0, sizeof(h));
    int64_t r = 1;
    int batch = 8;
    int status = LLP_OK;
    for (;;) {
        for (int i = 0; i < batch && r <= max_rounds; ++i, ++r)
            hipLaunchKernelGGL(k_jobs_level, dim3(a.nseg), dim3(JB), 0, st, a, (int)r);
        LLP_HIP(hipGetLastError());
        s = readback(st, a.ctrl, &h, sizeof(h));
        if (s) return s;
        if (h.status || h.done) break;
        if (o.abort_host && *o.abort_host) { status = LLP_E_ABORTED; break; }
        if (r > max_rounds) { status = LLP_E_NOT_CONVERGED; break; }
        if (batch < 64) batch *= 2;
    }
    if (status == LLP_OK && h.status == 0) hipLaunchKernelGGL(k_jobs_final, dim3(grid1(n)), dim3(256), 0, st, a);
    LLP_HIP(hipGetLastError());
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    s = readback(st, a.ctrl, &h, sizeof(h));
    if (s) return s;
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = h.rounds;
        o.stats->candidates = h.ready;
        o.stats->advances = h.ready;
        o.stats->edges_inspected = h.edges;
        o.stats->states_gathered = h.edges;
        if (timing) {
            float ms = 0.f;
            LLP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            o.stats->device_ms = ms;
        }
    }
    if (timing) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    if (h.diag[0])
        return fail(LLP_E_INPUT, "index guard %d fired: index %d bound %d context %d %d", h.diag[0], h.diag[1],
                    h.diag[2], h.diag[3], h.diag[4]);
    if (h.status == LLP_E_CYCLE) return fail(LLP_E_CYCLE, "the job arcs contain a cycle");
    if (h.status == LLP_E_OVERFLOW) return fail(LLP_E_OVERFLOW, "a completion time does not fit int32");
    if (h.status) return fail(h.status, "device status %d", h.status);
    if (status == LLP_E_NOT_CONVERGED) return fail(status, "not converged after %lld rounds", (long long)max_rounds);
    if (status == LLP_E_ABORTED) return fail(status, "aborted by the host flag");
    return LLP_OK;
}

}  // namespace llp

extern "C" int llp_solve_jobs(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx, const int32_t* dur,
                              const int32_t* succ_ptr, const int32_t* succ_idx, int32_t* start,
                              const llp_opts* opts) {
    return llp::solve_jobs(n, pred_ptr, pred_idx, dur, succ_ptr, succ_idx, start, opts);
}
