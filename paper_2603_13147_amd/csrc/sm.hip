// sm.hip - the LLP sweep for the man-optimal stable matching (paper Section
// 5.4) on gfx950.
//
// State.  G[m] is the index of the woman man m currently targets in his list
// (bottom 0, bound n - 1).  m is forbidden when his target is also targeted
// by a man she ranks better; alpha(G, m) = G[m] + 1.
//
// The forbidden test is answered by best[w], the smallest key that has ever
// targeted woman w, key = rank << 32 | man << 16 | index (64-bit atomicMin).
// The man holding best[w] targets w at every moment (he can only be moved on
// by a better key, which then holds w), so a man whose key loses the minimum
// at w is forbidden in the current state and may advance; a man whose key
// wins displaces the previous holder, who becomes forbidden.  (The predicate
// counts every man who has reached w in his list; from the bottom only the
// current holder matters, and a warm start registers the proposals its
// indices imply before the sweep.)  Because the
// displaced key carries its index, the displacing thread knows where the
// displaced man resumes without reading his G.
//
// Schedules (all reach the same least fixpoint):
//  - chains (default): one thread per man; a thread whose man is rejected
//    advances him and proposes again, a thread whose man displaces another
//    carries on with the displaced man, and a thread ends when its man lands
//    on a woman nobody held.  opts->chunk > 0 bounds the proposals a thread
//    makes per launch; a man still forbidden at the bound is parked and the
//    next launch (round) resumes him.
//  - dense rounds (LLP_SCHED_FIXED + LLP_DENSE): every round evaluates every
//    man once at his current target and advances the forbidden ones by one.
//  - random rounds (LLP_SCHED_RANDOM): dense rounds in which each forbidden
//    man advances only on a seeded coin flip.
#include <string.h>

#include "llp_dev.h"
#include "llp_host.h"

namespace llp {

constexpr unsigned long long SM_EMPTY = ~0ull;
constexpr int SM_NFLAG = 64;
constexpr int SM_LOOKAHEAD = 4;   // women examined per round trip of a chain

struct SCtrl {
    int done;
    int status;
    int last_round;
    int pad;
    int diag[8];
    long long proposals;
    int flag[SM_NFLAG];   // flag[r & 63]: round r left work for round r + 1
};

struct SArgs {
    int n;
    const short* mpref;   // [n * n] woman ids
    const short* wrank;   // [n * n] rank of man m for woman w
    int* G;               // proposal index per man
    unsigned long long* best;
    int* pend;            // round in which a parked man resumes (chunked chains)
    SCtrl* ctrl;
    const int* warm;      // warm start (nullable): man m has proposed to his first warm[m] women
    int chunk;            // proposals per thread per launch, 0 = unbounded
    int random;           // random rounds
    unsigned long long seed;
    int* combo;           // n <= SM_LDS_MAX: [n * SM_COMBO] w | rank of m for w << 16, by man and list position
};

__device__ __forceinline__ unsigned long long sm_key(int rank, int man, int idx) {
    return ((unsigned long long)(unsigned)rank << 32) | ((unsigned long long)(unsigned)man << 16) |
           (unsigned long long)(unsigned)idx;
}

__device__ __forceinline__ unsigned long long amin64(unsigned long long* p, unsigned long long v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_sm_init(SArgs a, const int* warm) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long i = tid; i < a.n; i += nt) {
        int g = 0;
        if (warm) {
            g = warm[i];
            if (g < 0 || g >= a.n) g = 0;
        }
        a.G[i] = g;
        a.best[i] = SM_EMPTY;
        a.pend[i] = 1;
    }
    if (tid == 0) memset(a.ctrl, 0, sizeof(SCtrl));
}

__device__ __forceinline__ int sm_warm(const SArgs& a, int m) {
    int g = a.warm[m];
    return (g < 0 || g >= a.n) ? 0 : g;
}

// Warm start: index G0[m] means man m has already proposed to the women
// before it (the predicate counts every man who has reached w in his list),
// so those proposals are registered before the sweep starts.
__global__ void k_sm_warm_register(SArgs a) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long m = tid; m < a.n; m += nt) {
        const int g0 = sm_warm(a, (int)m);
        for (int i = 0; i < g0; ++i) {
            int w = guard(a.mpref[m * a.n + i], a.n, a.ctrl->diag, 9, (int)m, i);
            int rk = guard(a.wrank[(long long)w * a.n + m], a.n, a.ctrl->diag, 10, w, (int)m);
            amin64(&a.best[w], sm_key(rk, (int)m, i));
        }
    }
}

// One workgroup per list (men's lists first, then women's rank rows): every
// row must be a permutation of 0..n-1.  n <= 32767, so a row's bitmap fits
// in 4 KB of LDS.
__global__ void k_sm_validate(SArgs a) {
    __shared__ unsigned bits[1024];
    const int row = blockIdx.x;
    const short* p = row < a.n ? a.mpref + (long long)row * a.n : a.wrank + (long long)(row - a.n) * a.n;
    const int words = (a.n + 31) >> 5;
    for (int i = threadIdx.x; i < words; i += blockDim.x) bits[i] = 0u;
    __syncthreads();
    bool bad = false;
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) {
        int x = p[i];
        if (x < 0 || x >= a.n) {
            bad = true;
            continue;
        }
        unsigned old = atomicOr(&bits[x >> 5], 1u << (x & 31));
        if (old & (1u << (x & 31))) bad = true;
    }
    if (bad) set_status(&a.ctrl->status, LLP_E_INPUT);
}

// Chains.  Launch r resumes the men whose pend stamp is r (round 1: all).
__global__ void k_sm_chain(SArgs a, int r) {
    SCtrl* c = a.ctrl;
    if (ld_relaxed(&c->done) || ld_relaxed(&c->status)) return;
    if (r > 1 && ld_relaxed(&c->flag[(r - 1) & (SM_NFLAG - 1)]) == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->done = 1;
            c->last_round = r - 1;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c->flag[(r + 1) & (SM_NFLAG - 1)] = 0;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    long long made = 0;
    if (t < a.n && a.pend[t] == r) {
        const int n = a.n;
        int m = t;
        int g = guard(a.G[m], n, c->diag, 8, m);
        const long long cap = a.chunk > 0 ? a.chunk : (long long)n * n + n;
        for (;;) {
            if (g >= n) {
                set_status(&c->status, LLP_E_INFEASIBLE);
                break;
            }
            if (made >= cap) {
                // park m, still to propose at index g, for the next launch
                amax(&a.G[m], g);
                a.pend[m] = r + 1;
                st_relaxed(&c->flag[r & (SM_NFLAG - 1)], 1);
                break;
            }
            // look ahead: the next women on m's list, their ranks of m and their
            // current best keys are independent loads; a woman whose best key
            // already beats m's rejects him without an atomic (best only
            // decreases), so a run of rejections costs one round trip
            const int la = (int)min((long long)SM_LOOKAHEAD, min((long long)(n - g), cap - made));
            int wv[SM_LOOKAHEAD];
            unsigned long long kv[SM_LOOKAHEAD], bv[SM_LOOKAHEAD];
#pragma unroll
            for (int i = 0; i < SM_LOOKAHEAD; ++i) {
                if (i < la) {
                    wv[i] = guard(a.mpref[(long long)m * n + g + i], n, c->diag, 1, m, g + i);
                } else {
                    wv[i] = 0;
                }
            }
#pragma unroll
            for (int i = 0; i < SM_LOOKAHEAD; ++i) {
                kv[i] = ~0ull;
                bv[i] = 0ull;
                if (i < la) {
                    int rk = guard(a.wrank[(long long)wv[i] * n + m], n, c->diag, 2, wv[i], m);
                    kv[i] = sm_key(rk, m, g + i);
                    bv[i] = a.best[wv[i]];
                }
            }
            int skip = 0;
#pragma unroll
            for (int i = 0; i < SM_LOOKAHEAD; ++i)
                if (skip == i && i < la && bv[i] < kv[i]) skip = i + 1;
            if (skip == la) {   // every looked-at woman holds a better man
                g += la;
                made += la;
                continue;
            }
            g += skip;
            made += skip + 1;
            int w = 0;
            unsigned long long key = 0;
#pragma unroll
            for (int i = 0; i < SM_LOOKAHEAD; ++i)
                if (i == skip) {
                    w = wv[i];
                    key = kv[i];
                }
            unsigned long long old = amin64(&a.best[w], key);
            if (old < key) {        // w holds a better man: m is forbidden
                ++g;
                continue;
            }
            amax(&a.G[m], g);       // m targets w and is not forbidden
            if (old == SM_EMPTY || old == key) break;
            // the previous holder is now forbidden at w: carry him on, unless
            // the key was registered for a warm start (he is already past w)
            m = guard((int)((old >> 16) & 0xffffull), n, c->diag, 3, w, (int)(old & 0xffff));
            g = (int)(old & 0xffffull) + 1;
            if (a.warm && g - 1 < sm_warm(a, m)) break;
        }
    }
    long long tot = wave_sum64(made);
    if (lane() == 0 && tot) atomicAdd((unsigned long long*)&c->proposals, (unsigned long long)tot);
}

// One workgroup runs every chain of a cold start with n <= SM_LDS_MAX:
// best[] and the proposal indices live in LDS, so the displacement atomic and
// the look-ahead's best-key reads stay on the CU (a chain's steps are
// dependent; across XCDs an atomic must reach the memory side).  Thread t
// starts men t, t + 1024, ... in turn and carries displaced men as above.
constexpr int SM_LDS_MAX = 12288;   // 12 B of LDS per man: 144 KB
constexpr int SM_COMBO = 64;        // list positions per man held as (woman, rank) pairs
constexpr int SM_LDS_LOOKAHEAD = 6;   // women examined per round trip of a chain in k_sm_lds
constexpr int SM_LDS_THREADS = 1024;

// The i-th woman w on m's list and her rank of m, as w | rank << 16.
__device__ __forceinline__ int sm_pair(const SArgs& a, int m, int i) {
    const int n = a.n;
    const int w = guard(a.mpref[(long long)m * n + i], n, a.ctrl->diag, 4, m, i);
    const int rk = guard(a.wrank[(long long)w * n + m], n, a.ctrl->diag, 5, w, m);
    return w | (rk << 16);
}

// combo[m * SM_COMBO + i] = sm_pair(m, i) for the first SM_COMBO positions of
// every list (men make about log n proposals on average): a chain step there
// reads one entry (woman and her rank of m together) instead of a list entry
// and then a rank; later positions read both.  One thread per entry.
__global__ void k_sm_combo(SArgs a) {
    const int n = a.n;
    const int k = min(n, SM_COMBO);
    const long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (x >= (long long)n * k) return;
    const int m = (int)(x / k), i = (int)(x % k);
    a.combo[(long long)m * SM_COMBO + i] = sm_pair(a, m, i);
}

__global__ void __launch_bounds__(SM_LDS_THREADS) k_sm_lds(SArgs a) {
    __shared__ unsigned long long best[SM_LDS_MAX];
    __shared__ int gl[SM_LDS_MAX];
    SCtrl* c = a.ctrl;
    const int n = a.n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        best[i] = SM_EMPTY;
        gl[i] = 0;
    }
    __syncthreads();
    long long made = 0;
    bool infeasible = false;
    for (int t = threadIdx.x; t < n && !infeasible; t += blockDim.x) {
        int m = t, g = 0;
        for (;;) {
            if (g >= n) {
                infeasible = true;
                break;
            }
            const int la = min(SM_LDS_LOOKAHEAD, n - g);
            int wv[SM_LDS_LOOKAHEAD], cw[SM_LDS_LOOKAHEAD];
            unsigned long long kv[SM_LDS_LOOKAHEAD], bv[SM_LDS_LOOKAHEAD];
            if (g + SM_LDS_LOOKAHEAD <= SM_COMBO) {   // the whole look-ahead window is in the table
#pragma unroll
                for (int i = 0; i < SM_LDS_LOOKAHEAD; ++i) cw[i] = i < la ? a.combo[(long long)m * SM_COMBO + g + i] : 0;
            } else {
#pragma unroll
                for (int i = 0; i < SM_LDS_LOOKAHEAD; ++i)
                    cw[i] = i >= la ? 0 : g + i < SM_COMBO ? a.combo[(long long)m * SM_COMBO + g + i] : sm_pair(a, m, g + i);
            }
#pragma unroll
            for (int i = 0; i < SM_LDS_LOOKAHEAD; ++i) {
                wv[i] = cw[i] & 0xffff;   // < n: sm_pair guarded it
                kv[i] = ~0ull;
                bv[i] = 0ull;
                if (i < la) {
                    kv[i] = sm_key(cw[i] >> 16, m, g + i);
                    bv[i] = best[wv[i]];
                }
            }
            int skip = 0;
#pragma unroll
            for (int i = 0; i < SM_LDS_LOOKAHEAD; ++i)
                if (skip == i && i < la && bv[i] < kv[i]) skip = i + 1;
            if (skip == la) {
                g += la;
                made += la;
                continue;
            }
            g += skip;
            made += skip + 1;
            int w = 0;
            unsigned long long key = 0;
#pragma unroll
            for (int i = 0; i < SM_LDS_LOOKAHEAD; ++i)
                if (i == skip) {
                    w = wv[i];
                    key = kv[i];
                }
            const unsigned long long old = atomicMin(&best[w], key);
            if (old < key) {
                ++g;
                continue;
            }
            atomicMax(&gl[m], g);
            if (old == SM_EMPTY || old == key) break;
            m = guard((int)((old >> 16) & 0xffffull), n, c->diag, 3, w, (int)(old & 0xffff));
            g = (int)(old & 0xffffull) + 1;
        }
    }
    if (infeasible) set_status(&c->status, LLP_E_INFEASIBLE);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) a.G[i] = gl[i];
    const long long tot = wave_sum64(made);
    if (lane() == 0 && tot) atomicAdd((unsigned long long*)&c->proposals, (unsigned long long)tot);
    if (threadIdx.x == 0) {
        c->done = 1;
        c->last_round = 1;
    }
}

__device__ __forceinline__ unsigned long long sm_mix(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Dense round r: every man registers his current proposal and advances by one
// if it loses (on a coin flip for random rounds).
__global__ void k_sm_round(SArgs a, int r) {
    SCtrl* c = a.ctrl;
    if (ld_relaxed(&c->done) || ld_relaxed(&c->status)) return;
    if (r > 1 && ld_relaxed(&c->flag[(r - 1) & (SM_NFLAG - 1)]) == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->done = 1;
            c->last_round = r - 1;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c->flag[(r + 1) & (SM_NFLAG - 1)] = 0;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.n;
    long long tot = wave_sum64(m < n ? 1 : 0);
    if (lane() == 0 && tot) atomicAdd((unsigned long long*)&c->proposals, (unsigned long long)tot);
    if (m >= n) return;
    int g = guard(a.G[m], n, c->diag, 7, m);
    int w = guard(a.mpref[(long long)m * n + g], n, c->diag, 4, m, g);
    int rk = guard(a.wrank[(long long)w * n + m], n, c->diag, 5, w, m);
    unsigned long long key = sm_key(rk, m, g);
    unsigned long long old = amin64(&a.best[w], key);
    // m displaced the previous holder, who is now forbidden: he finds out by
    // re-registering in the next round
    if (old != SM_EMPTY && old > key) st_relaxed(&c->flag[r & (SM_NFLAG - 1)], 1);
    if (old < key) {
        // forbidden: any later round also sees it (best[w] only decreases)
        st_relaxed(&c->flag[r & (SM_NFLAG - 1)], 1);
        bool go = true;
        if (a.random) go = (sm_mix(a.seed ^ ((unsigned long long)r << 32) ^ (unsigned)m) & 1ull) != 0;
        if (go) {
            if (g + 1 >= n) set_status(&c->status, LLP_E_INFEASIBLE);
            else a.G[m] = g + 1;
        }
    }
}

__global__ void k_sm_decode(SArgs a, int* wife) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long m = tid; m < a.n; m += nt) {
        int g = guard(a.G[m], a.n, a.ctrl->diag, 6, (int)m);
        wife[m] = a.mpref[m * a.n + g];
    }
}

// --------------------------------------------------------------- host
static size_t sm_ws(int64_t n, SArgs* a, char* base, size_t cap) {
    Carver cv{base, cap, 0, base == nullptr};
    unsigned long long* best = cv.take<unsigned long long>(n);
    int* G = cv.take<int>(n);
    int* pend = cv.take<int>(n);
    SCtrl* ctrl = cv.take<SCtrl>(1);
    int* combo = cv.take<int>(n <= SM_LDS_MAX ? (size_t)n * SM_COMBO : 0);
    if (a) {
        a->combo = combo;
        a->best = best;
        a->G = G;
        a->pend = pend;
        a->ctrl = ctrl;
    }
    return cv.used;
}

size_t sm_workspace_bytes(int64_t n) { return sm_ws(n, nullptr, nullptr, 0); }

static int grid_for(int64_t work, int block) {
    int64_t g = (work + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 65535 * 4 ? 65535 * 4 : g));
}

int solve_sm(int32_t n, const int16_t* men_pref, const int16_t* women_rank, int32_t* wife,
             int32_t* proposal_idx, const llp_opts* opts) {
    if (n <= 0 || n > 32767) return fail(LLP_E_ARG, "n must be in [1, 32767] (got %d)", n);
    if (!men_pref || !women_rank || !wife) return fail(LLP_E_ARG, "men_pref, women_rank and wife are required");
    llp_opts o = opts_or_default(opts);
    if (o.sched > LLP_SCHED_RANDOM) return fail(LLP_E_ARG, "unknown schedule %u", o.sched);
    if (o.sched == LLP_SCHED_LEARNED || o.sched == LLP_SCHED_HYBRID)
        return fail(LLP_E_ARG, "stable marriage supports the plain, fixed and random schedules");
    if (o.chunk < 0) return fail(LLP_E_ARG, "chunk must be >= 0");
    hipStream_t st = (hipStream_t)o.stream;
    SArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.mpref = men_pref;
    a.wrank = women_rank;
    a.chunk = o.chunk;
    a.random = o.sched == LLP_SCHED_RANDOM;
    a.seed = o.seed;
    a.warm = o.warm_start;
    const bool rounds = a.random || (o.sched == LLP_SCHED_FIXED && (o.flags & LLP_DENSE));

    size_t need = sm_ws(n, nullptr, nullptr, 0);
    void* ws = nullptr;
    int s = get_workspace(o, need, &ws);
    if (s) return s;
    sm_ws(n, &a, (char*)ws, need);
    if (proposal_idx) a.G = proposal_idx;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    const int blk = 64;
    hipLaunchKernelGGL(k_sm_init, dim3(grid_for(n, 256)), dim3(256), 0, st, a, o.warm_start);
    if (o.flags & LLP_VALIDATE) hipLaunchKernelGGL(k_sm_validate, dim3(2 * n), dim3(256), 0, st, a);
    if (a.warm) hipLaunchKernelGGL(k_sm_warm_register, dim3(grid_for(n, 64)), dim3(64), 0, st, a);
    LLP_HIP(hipGetLastError());

    // Unbounded chains finish in one launch; chunked chains and dense rounds
    // need at most n * n proposals in all, hence the default round limit.
    const int64_t max_rounds = o.max_rounds > 0 ? o.max_rounds : (int64_t)n * n + 2;
    SCtrl h;
    memset(&h, 0, sizeof(h));
    int64_t r = 1;
    int batch = rounds || a.chunk > 0 ? 8 : 2;
    int status = LLP_OK;
    const bool lds = !rounds && a.chunk == 0 && !a.warm && n <= SM_LDS_MAX;
    if (lds) {
        const long long entries = (long long)n * (n < SM_COMBO ? n : SM_COMBO);
        hipLaunchKernelGGL(k_sm_combo, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, a);
        hipLaunchKernelGGL(k_sm_lds, dim3(1), dim3(SM_LDS_THREADS), 0, st, a);
        ++r;
    }
    while (!lds) {
        for (int i = 0; i < batch && r <= max_rounds; ++i, ++r) {
            if (rounds) hipLaunchKernelGGL(k_sm_round, dim3(grid_for(n, blk)), dim3(blk), 0, st, a, (int)r);
            else hipLaunchKernelGGL(k_sm_chain, dim3(grid_for(n, blk)), dim3(blk), 0, st, a, (int)r);
        }
        LLP_HIP(hipGetLastError());
        s = readback(st, a.ctrl, &h, sizeof(h));
        if (s) return s;
        if (h.status || h.done) break;
        if (o.abort_host && *o.abort_host) { status = LLP_E_ABORTED; break; }
        if (r > max_rounds) { status = LLP_E_NOT_CONVERGED; break; }
        if (batch < 64) batch *= 2;
    }
    hipLaunchKernelGGL(k_sm_decode, dim3(grid_for(n, 256)), dim3(256), 0, st, a, wife);
    LLP_HIP(hipGetLastError());
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    s = readback(st, a.ctrl, &h, sizeof(h));
    if (s) return s;
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = h.done ? h.last_round : (r - 1);
        o.stats->candidates = h.proposals;
        o.stats->advances = h.proposals;
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
    if (h.status == LLP_E_INPUT) return fail(LLP_E_INPUT, "a preference list is not a permutation of 0..n-1");
    if (h.status == LLP_E_INFEASIBLE) return fail(LLP_E_INFEASIBLE, "a man exhausted his list (malformed lists)");
    if (h.status) return fail(h.status, "device status %d", h.status);
    if (status == LLP_E_NOT_CONVERGED) return fail(status, "not converged after %lld rounds", (long long)max_rounds);
    if (status == LLP_E_ABORTED) return fail(status, "aborted by the host flag");
    return LLP_OK;
}

}  // namespace llp

extern "C" int llp_solve_sm(int32_t n, const int16_t* men_pref, const int16_t* women_rank, int32_t* wife,
                            int32_t* proposal_idx, const llp_opts* opts) {
    return llp::solve_sm(n, men_pref, women_rank, wife, proposal_idx, opts);
}
