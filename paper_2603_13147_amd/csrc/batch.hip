// batch.hip - workgroup-local LLP sweeps: the 0-1 knapsack (paper Section
// 5.8), small SSSP instances, and the batched persistent solve that mixes
// thousands of them in one launch, with its hipGraph replay and autotuner.
//
// Knapsack.  Cell (k, c) of the DP table is forbidden below
// max(G[k-1][c], v_k + G[k-1][c - w_k]); once row k-1 is final every cell of
// row k is forbidden exactly until it takes that value, so the workgroup
// advances a whole row per step.  Thread t keeps cells c = t + i*T (i < CH) of
// the current row in registers; per item the row is published to LDS, one
// barrier, and every thread reads the shifted cells c - w_k it needs.  With
// room for two LDS rows the buffers alternate and one barrier per item
// suffices; otherwise a second barrier protects the single buffer.  Items
// heavier than W or worth nothing leave the row unchanged and are skipped.
//
// Small SSSP.  State G[v] = INF - d(v) in LDS (bottom 0, the source INF) and
// two frontier bitmaps.  Each round every vertex whose bit is set pushes
// single-arc partial advances G[x] <- max(G[x], G[u] - w) along its out-arcs
// with LDS atomicMax (Definition 3: a partial maximum is an alpha-forbidden
// advance), marking the advanced vertices for the next round, until a round
// advances nothing.
//
// Batch.  A persistent grid; each workgroup claims `chunk` consecutive
// instances from a device queue counter and solves them one after another.
// Every instance's ranges are checked against the pool sizes before any of
// its words are read.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "llp_dev.h"
#include "llp_host.h"

namespace llp {

constexpr int KN_MAX_W = 16383;

// Largest workgroup a kernel holding CH row cells per thread in registers is
// built for (16384 cells per workgroup keeps the register budget).
constexpr int ch_max_block(int ch) { return 16384 / ch > 1024 ? 1024 : 16384 / ch; }
constexpr int SS_MAX_N = 8192;
constexpr size_t BATCH_STATIC_LDS = 64;   // bytes of k_batch's static LDS (claim word, flags), rounded up

struct BCtrl {
    int head;          // queue: next unclaimed instance
    int status;        // first nonzero instance status
    int max_w;         // limits measured over desc
    int max_n;
    int bad_kind;
    int pad[3];
};

// --------------------------------------------------------------- knapsack
// Solve one knapsack instance with the calling workgroup.  buf0 / buf1: LDS
// rows of W + 1 ints (buf1 == nullptr: single buffer).  Requires
// CH * blockDim.x >= W + 1.  Returns the status (uniform); the best value is
// written to *best (thread owning cell W), the last row to row (nullable).
template <int CH>
__device__ int knap_wg(const int* wt, const int* val, int items, int W, int* buf0, int* buf1, int* best,
                       int* row) {
    const int T = blockDim.x, t = threadIdx.x;
    int g[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) g[i] = 0;
    int st = LLP_OK;
    bool ovf = false;
    int par = 0;
    for (int k = 0; k < items; ++k) {
        const int w = wt[k], v = val[k];
        if (w < 0 || v < 0) {
            st = LLP_E_INPUT;
            break;
        }
        if (w > W || v == 0) continue;
        int* buf = (buf1 && par) ? buf1 : buf0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            int c = t + i * T;
            if (c <= W) buf[c] = g[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            int c = t + i * T;
            if (c <= W && c >= w) {
                int y = buf[c - w];
                if (y > LLP_INF - v) ovf = true;
                else g[i] = max(g[i], y + v);
            }
        }
        if (!buf1) __syncthreads();
        par ^= 1;
    }
    if (__syncthreads_or(ovf) && st == LLP_OK) st = LLP_E_OVERFLOW;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        int c = t + i * T;
        if (c <= W) {
            if (row) row[c] = g[i];
            if (c == W && best) *best = g[i];
        }
    }
    return st;
}

// --------------------------------------------------------------- small SSSP
// Solve one SSSP instance (out-CSR) with the calling workgroup.  G: LDS
// int[n]; cur, nxt: LDS bitmaps of ceil(n/32) words; ptr: LDS int[n + 1],
// filled from gptr; fl: LDS int[4].  dist: output int[n].  Returns the
// status (uniform).
__device__ int sssp_wg(const int* gptr, const int* dst, const int* wgt, int n, int m, int src, int* G,
                       unsigned* cur, unsigned* nxt, int* ptr, int* fl, int* dist, int max_rounds,
                       int* rounds_out) {
    const int T = blockDim.x, t = threadIdx.x;
    const int words = (n + 31) >> 5;
    for (int v = t; v < n; v += T) G[v] = (v == src) ? LLP_INF : 0;
    for (int v = t; v <= n; v += T) ptr[v] = gptr[v];   // row offsets held in LDS for every round
    for (int i = t; i < words; i += T) {
        cur[i] = (i == (src >> 5)) ? (1u << (src & 31)) : 0u;
        nxt[i] = 0u;
    }
    if (t < 4) fl[t] = 0;   // fl[0], fl[1]: advanced in round parity; fl[2]: bad input; fl[3]: overflow
    __syncthreads();
    int r = 0;
    for (;; ++r) {
        if (r >= max_rounds) break;
        bool adv = false, bad = false, ovf = false;
        for (int u = t; u < n; u += T) {
            if (!(cur[u >> 5] & (1u << (u & 31)))) continue;
            int b = ptr[u], e = ptr[u + 1];
            if (b < 0 || e > m || e < b) {
                bad = true;
                continue;
            }
            const int gu = G[u];
            for (int k0 = b; k0 < e; k0 += 8) {
                // the arcs' loads are all issued before any is checked
                int xs[8], ws[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = k0 + j < e ? k0 + j : b;
                    xs[j] = dst[k];
                    ws[j] = wgt[k];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (k0 + j >= e) break;
                    const int x = xs[j], w = ws[j];
                    if ((unsigned)x >= (unsigned)n || w < 0) {
                        bad = true;
                        continue;
                    }
                    int cand = gu - w;
                    if (cand <= 0) {
                        ovf = true;
                        continue;
                    }
                    if (cand > G[x]) {
                        int old = atomicMax(&G[x], cand);
                        if (old < cand) {
                            atomicOr(&nxt[x >> 5], 1u << (x & 31));
                            adv = true;
                        }
                    }
                }
            }
        }
        if (adv) fl[r & 1] = 1;
        if (bad) fl[2] = 1;
        if (ovf) fl[3] = 1;
        __syncthreads();
        const bool more = fl[r & 1] != 0 && fl[2] == 0;
        // clear the bitmap the next round fills and the next round's flag
        for (int i = t; i < words; i += T) cur[i] = 0u;
        if (t == 0) fl[(r + 1) & 1] = 0;
        __syncthreads();
        unsigned* tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (!more) {
            ++r;
            break;
        }
    }
    int st = LLP_OK;
    if (fl[2]) st = LLP_E_INPUT;
    else if (r >= max_rounds && fl[(r - 1) & 1]) st = LLP_E_NOT_CONVERGED;
    // overflow: an unreached vertex with a reached in-neighbour
    if (st == LLP_OK && fl[3]) {
        bool o = false;
        for (int u = t; u < n; u += T) {
            if (G[u] <= 0) continue;
            for (int k = max(ptr[u], 0); k < min(ptr[u + 1], m); ++k) {
                int x = dst[k];
                if ((unsigned)x < (unsigned)n && G[x] == 0) o = true;
            }
        }
        if (__syncthreads_or(o)) st = LLP_E_OVERFLOW;
    }
    for (int v = t; v < n; v += T) {
        int g = G[v];
        dist[v] = g > 0 ? LLP_INF - g : LLP_INF;
    }
    if (rounds_out && t == 0) *rounds_out = r;
    return st;
}

// --------------------------------------------------------------- kernels
template <int CH>
__global__ void __launch_bounds__(ch_max_block(CH)) k_knapsack_one(const int* wt, const int* val, int items, int W, int dbuf,
                                                      int* best, int* row, int* status) {
    extern __shared__ int lds[];
    int st = knap_wg<CH>(wt, val, items, W, lds, dbuf ? lds + (W + 1) : nullptr, best, row);
    if (threadIdx.x == 0) *status = st;
}

struct BArgs {
    int count;
    const llp_instance* desc;
    const int* pool;
    long long pool_words;
    int* out_pool;
    long long out_words;
    int* out_status;
    BCtrl* ctrl;
    int chunk;
    const int* order;   // claim order (instance ids)
    int kn_w;        // LDS row capacity - 1 (max W this launch supports)
    int kn_dbuf;
    int ss_n;        // max SSSP n this launch supports
};

__device__ __forceinline__ bool in_range(long long off, long long len, long long total) {
    return off >= 0 && len >= 0 && off <= total && len <= total - off;
}

template <int CH>
__device__ void batch_one(const BArgs& a, int i, int* lds, int* sfl) {
    const llp_instance d = a.desc[i];
    int st = LLP_OK;
    if (d.kind == LLP_KIND_KNAPSACK) {
        const int items = d.n, W = d.cap_or_source;
        if (items < 0 || W < 0 || W > a.kn_w || W + 1 > CH * (int)blockDim.x ||
            !in_range(d.in_off, 2ll * items, a.pool_words) || !in_range(d.out_off, 1, a.out_words)) {
            st = LLP_E_INPUT;
        } else {
            const int* wt = a.pool + d.in_off;
            st = knap_wg<CH>(wt, wt + items, items, W, lds, a.kn_dbuf ? lds + (a.kn_w + 1) : nullptr,
                             a.out_pool + d.out_off, nullptr);
        }
    } else if (d.kind == LLP_KIND_SSSP) {
        const int n = d.n, src = d.cap_or_source;
        const long long m = d.m;
        if (n < 1 || n > a.ss_n || src < 0 || src >= n || m < 0 || m > 0x7fffffffll ||
            !in_range(d.in_off, (long long)n + 1 + 2 * m, a.pool_words) || !in_range(d.out_off, n, a.out_words)) {
            st = LLP_E_INPUT;
        } else {
            const int* ptr = a.pool + d.in_off;
            const int* dst = ptr + n + 1;
            const int* wgt = dst + m;
            const int words = (n + 31) >> 5;
            int* G = lds;
            unsigned* cur = (unsigned*)(lds + a.ss_n);
            unsigned* nxt = cur + ((a.ss_n + 31) >> 5);
            int* lptr = (int*)(nxt + ((a.ss_n + 31) >> 5));
            st = sssp_wg(ptr, dst, wgt, n, (int)m, src, G, cur, nxt, lptr, sfl, a.out_pool + d.out_off, n + 2,
                         nullptr);
            (void)words;
        }
    } else {
        st = LLP_E_INPUT;
    }
    if (threadIdx.x == 0) {
        if (a.out_status) a.out_status[i] = st;
        if (st) set_status(&a.ctrl->status, st);
    }
    __syncthreads();   // LDS is reused by the next instance
}

template <int CH>
__global__ void __launch_bounds__(ch_max_block(CH)) k_batch(BArgs a) {
    extern __shared__ int lds[];
    __shared__ int claim;
    __shared__ int sfl[4];
    for (;;) {
        if (threadIdx.x == 0) claim = atomicAdd(&a.ctrl->head, a.chunk);
        __syncthreads();
        const int i0 = claim;
        __syncthreads();
        if (i0 >= a.count) break;
        const int i1 = min(i0 + a.chunk, a.count);
        for (int i = i0; i < i1; ++i) {
            const int j = a.order[i];   // uniform in the workgroup
            if ((unsigned)j >= (unsigned)a.count) {
                if (threadIdx.x == 0) set_status(&a.ctrl->status, LLP_E_HIP);
                continue;
            }
            batch_one<CH>(a, j, lds, sfl);
        }
    }
}

// Claim order, rebuilt on the device by every solve and every graph replay:
// longest estimated cost first (longest-processing-time order), so the last
// instances to start are the short ones.  Estimated cost: knapsack cells, or
// 20 per SSSP arc (the ratio of the two measured per unit on this batch
// kernel).  A one-workgroup counting sort over 256 cost classes (four per
// octave), costliest class first; order within a class is arbitrary.
constexpr int ORD_CLASSES = 256;

__device__ __forceinline__ int cost_slot(const llp_instance& d) {
    long long c = 0;
    if (d.kind == LLP_KIND_KNAPSACK) c = (long long)max(d.n, 0) * (max(d.cap_or_source, 0) + 1);
    else if (d.kind == LLP_KIND_SSSP) c = 20 * (d.m > 0 ? d.m : 0ll) + max(d.n, 0);
    if (c <= 0) return ORD_CLASSES - 1;
    const int e = 63 - __clzll((unsigned long long)c);
    const int f = e >= 2 ? (int)((c >> (e - 2)) & 3) : (int)((c << (2 - e)) & 3);
    return ORD_CLASSES - 1 - (4 * e + f);   // 4 e + f <= 251
}

__global__ void __launch_bounds__(1024) k_batch_order(const llp_instance* desc, int count, int* order) {
    __shared__ int cnt[ORD_CLASSES];
    const int t = threadIdx.x, T = blockDim.x;
    for (int i = t; i < ORD_CLASSES; i += T) cnt[i] = 0;
    __syncthreads();
    for (int i = t; i < count; i += T) atomicAdd(&cnt[cost_slot(desc[i])], 1);
    __syncthreads();
    if (t < 64) {
        // exclusive scan of the class counts, four classes per lane
        int v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = cnt[4 * t + j];
            sum += v[j];
        }
        int run = wave_incl_sum(sum) - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cnt[4 * t + j] = run;
            run += v[j];
        }
    }
    __syncthreads();
    for (int i = t; i < count; i += T) order[atomicAdd(&cnt[cost_slot(desc[i])], 1)] = i;
}

// queue reset (a fill kernel, so the launch can be captured in a graph)
__global__ void k_batch_reset(BCtrl* c, int* status_dev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->head = 0;
        c->status = 0;
        if (status_dev) *status_dev = 0;
    }
}

__global__ void k_batch_status(const BCtrl* c, int* status_dev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status_dev = c->status;
}

// limits over desc: largest knapsack W, largest SSSP n, unknown kinds
__global__ void k_batch_limits(const llp_instance* desc, int count, BCtrl* c) {
    int mw = 0, mn = 0, bad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        llp_instance d = desc[i];
        if (d.kind == LLP_KIND_KNAPSACK) mw = max(mw, d.cap_or_source);
        else if (d.kind == LLP_KIND_SSSP) mn = max(mn, d.n);
        else bad = 1;
    }
    mw = wave_max(mw);
    mn = wave_max(mn);
    const bool anybad = __any(bad);
    if (lane() == 0) {
        atomicMax(&c->max_w, mw);
        atomicMax(&c->max_n, mn);
        if (anybad) atomicMax(&c->bad_kind, 1);
    }
}

__global__ void k_batch_limits_reset(BCtrl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        BCtrl z;
        memset(&z, 0, sizeof(z));
        *c = z;
    }
}

// --------------------------------------------------------------- host
static const int CH_OPTS[] = {4, 8, 16, 32};

static int pick_ch(int W, int T) {
    for (int ch : CH_OPTS)
        if ((long long)ch * T >= (long long)W + 1 && T <= ch_max_block(ch)) return ch;
    return 0;
}

template <class F>
static int dispatch_ch(int ch, F&& f) {
    switch (ch) {
        case 4: return f(std::integral_constant<int, 4>());
        case 8: return f(std::integral_constant<int, 8>());
        case 16: return f(std::integral_constant<int, 16>());
        case 32: return f(std::integral_constant<int, 32>());
        default: return fail(LLP_E_ARG, "no kernel for %d cells per thread", ch);
    }
}

static size_t lds_limit() {
    size_t l = device_info().lds_per_block;
    return l ? l : 65536;
}

int solve_knapsack(int32_t items, int32_t W, const int32_t* wt, const int32_t* val, int32_t* best,
                   int32_t* last_row, const llp_opts* opts) {
    if (items < 0) return fail(LLP_E_ARG, "items must be >= 0 (got %d)", items);
    if (W < 0 || W > KN_MAX_W) return fail(LLP_E_ARG, "W must be in [0, %d] (got %d)", KN_MAX_W, W);
    if (!best) return fail(LLP_E_ARG, "best is required");
    if (items > 0 && (!wt || !val)) return fail(LLP_E_ARG, "wt and val are required");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    int T = o.block > 0 ? o.block : 1024;
    if (T % 64 != 0 || T > 1024) return fail(LLP_E_ARG, "block must be a multiple of 64 up to 1024");
    const int ch = pick_ch(W, T);
    if (!ch) return fail(LLP_E_ARG, "W = %d needs more than 32 cells per thread at %d threads", W, T);
    const size_t row_bytes = (size_t)(W + 1) * 4;
    const int dbuf = 2 * row_bytes <= lds_limit();
    const size_t lds = dbuf ? 2 * row_bytes : row_bytes;
    if (lds > lds_limit()) return fail(LLP_E_ARG, "a row of W = %d does not fit in LDS", W);
    size_t need = 256;
    void* ws = nullptr;
    int s = get_workspace(o, need, &ws);
    if (s) return s;
    int* status = (int*)ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    s = dispatch_ch(ch, [&](auto c) {
        constexpr int CH = decltype(c)::value;
        if (lds > 65536) (void)hipFuncSetAttribute((const void*)k_knapsack_one<CH>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(k_knapsack_one<CH>, dim3(1), dim3(T), lds, st, wt, val, items, W, dbuf, best,
                           last_row, status);
        return hip_check(hipGetLastError(), "k_knapsack_one");
    });
    if (s) return s;
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    if (o.flags & LLP_ASYNC) {
        if (o.status_dev) LLP_HIP(hipMemcpyAsync(o.status_dev, status, 4, hipMemcpyDeviceToDevice, st));
        return LLP_OK;
    }
    int h = 0;
    s = readback(st, status, &h, sizeof(h));
    if (s) return s;
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = items;
        o.stats->advances = (int64_t)items * (W + 1);
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
    if (h == LLP_E_INPUT) return fail(h, "negative weight or value");
    if (h == LLP_E_OVERFLOW) return fail(h, "a DP value does not fit int32");
    if (h) return fail(h, "device status %d", h);
    return LLP_OK;
}

// ---------------------------------------------------------------- batch
static std::mutex g_bmu;

struct BatchPlan {
    int block, chunk, ch;
    int kn_w, kn_dbuf, ss_n;
    size_t lds;
};

// Workspace: the control block, then the claim order (int32[count]).
static size_t batch_bytes(int64_t count) { return 256 + (size_t)(count > 0 ? count : 0) * 4; }

static int batch_ws(void** ws, const llp_opts& o, int64_t count) { return get_workspace(o, batch_bytes(count), ws); }

size_t batch_workspace_bytes(int64_t count) { return batch_bytes(count); }

// Measure the limits over desc (one readback) and choose the launch shape.
static int batch_plan(int32_t count, const llp_instance* desc, const llp_opts& o, BCtrl* ctrl, BatchPlan* p) {
    hipStream_t st = (hipStream_t)o.stream;
    hipLaunchKernelGGL(k_batch_limits_reset, dim3(1), dim3(64), 0, st, ctrl);
    int g = (count + 255) / 256;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_batch_limits, dim3(g), dim3(256), 0, st, desc, count, ctrl);
    LLP_HIP(hipGetLastError());
    BCtrl h;
    int s = readback(st, ctrl, &h, sizeof(h));
    if (s) return s;
    if (h.bad_kind) return fail(LLP_E_ARG, "desc holds an instance kind other than knapsack or SSSP");
    if (h.max_w > KN_MAX_W) return fail(LLP_E_ARG, "a knapsack instance has W = %d > %d", h.max_w, KN_MAX_W);
    if (h.max_n > SS_MAX_N) return fail(LLP_E_ARG, "an SSSP instance has n = %d > %d", h.max_n, SS_MAX_N);
    int block = o.block, chunk = o.chunk;
    bool tuned_block = false;
    if (block <= 0 || chunk <= 0) {
        // the autotuner's record for this batch's size class (or the nearest)
        int tb = 0, tc = 0;
        if (tune_lookup(LLP_KIND_BATCH, count, &tb, &tc)) {
            if (block <= 0) {
                block = tb;
                tuned_block = true;
            }
            if (chunk <= 0) chunk = tc;
        }
    }
    if (block <= 0) block = 512;   // the autotuner's usual choice on the mixed batch
    if (chunk <= 0) chunk = 1;
    if (block % 64 != 0 || block > 1024) return fail(LLP_E_ARG, "block must be a multiple of 64 up to 1024");
    // a record is keyed by the instance count only: when its workgroup is too
    // small for this batch's widest knapsack row, 512 threads hold any W up
    // to KN_MAX_W
    if (tuned_block && !pick_ch(h.max_w, block)) block = 512;
    p->block = block;
    p->chunk = chunk;
    p->ch = pick_ch(h.max_w, block);
    if (!p->ch) return fail(LLP_E_ARG, "W = %d needs more than 32 cells per thread at %d threads", h.max_w, block);
    p->kn_w = h.max_w;
    p->ss_n = h.max_n > 0 ? h.max_n : 1;
    const size_t row = (size_t)(p->kn_w + 1) * 4;
    // SSSP: state, two frontier bitmaps and the row offsets
    const size_t ss = (size_t)p->ss_n * 4 + 2 * (size_t)((p->ss_n + 31) / 32) * 4 + (size_t)(p->ss_n + 1) * 4;
    size_t need1 = row > ss ? row : ss;
    size_t need2 = 2 * row > ss ? 2 * row : ss;
    // k_batch's own LDS (the claim word and the solver flags) comes first
    const size_t lim = lds_limit() - BATCH_STATIC_LDS;
    p->kn_dbuf = need2 <= lim;
    p->lds = p->kn_dbuf ? need2 : need1;
    if (p->lds > lim) return fail(LLP_E_ARG, "instances need %zu bytes of LDS", p->lds);
    return LLP_OK;
}

static int batch_grid(const BatchPlan& p, int count) {
    // resident workgroups: four per CU when LDS allows
    const size_t lim = 160 * 1024;
    int per_cu = (int)(lim / (p.lds + 1024));
    int by_threads = 2048 / p.block;
    if (per_cu > by_threads) per_cu = by_threads;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    long long g = (long long)device_info().cus * per_cu;
    long long need = (count + p.chunk - 1) / p.chunk;
    if (g > need) g = need;
    return (int)(g < 1 ? 1 : g);
}

static int batch_enqueue(const BatchPlan& p, int32_t count, const llp_instance* desc, const int32_t* pool,
                         int64_t pool_words, int32_t* out_pool, int64_t out_words, int32_t* out_status, BCtrl* ctrl,
                         hipStream_t st, int32_t* status_dev) {
    BArgs a;
    memset(&a, 0, sizeof(a));
    a.count = count;
    a.desc = desc;
    a.pool = pool;
    a.pool_words = pool_words;
    a.out_pool = out_pool;
    a.out_words = out_words;
    a.out_status = out_status;
    a.ctrl = ctrl;
    a.order = (const int*)((const char*)ctrl + 256);
    a.chunk = p.chunk;
    a.kn_w = p.kn_w;
    a.kn_dbuf = p.kn_dbuf;
    a.ss_n = p.ss_n;
    // limits and claim order are measured again by every launch sequence, so a
    // captured graph stays valid whatever else uses the workspace between
    // replays, and its replays see the current instance table
    const int lg = std::min(std::max((count + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(k_batch_limits_reset, dim3(1), dim3(64), 0, st, ctrl);
    hipLaunchKernelGGL(k_batch_limits, dim3(lg), dim3(256), 0, st, desc, count, ctrl);
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, st, desc, count, (int*)a.order);
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, ctrl, (int*)nullptr);
    const int grid = batch_grid(p, count);
    int s = dispatch_ch(p.ch, [&](auto c) {
        constexpr int CH = decltype(c)::value;
        if (p.lds > 65536) (void)hipFuncSetAttribute((const void*)k_batch<CH>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
        hipLaunchKernelGGL(k_batch<CH>, dim3(grid), dim3(p.block), p.lds, st, a);
        return hip_check(hipGetLastError(), "k_batch");
    });
    if (s) return s;
    if (status_dev) hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(64), 0, st, ctrl, status_dev);
    return hip_check(hipGetLastError(), "k_batch_status");
}

static int batch_args(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                      int32_t* out_pool, int64_t out_words) {
    if (count < 0) return fail(LLP_E_ARG, "count must be >= 0");
    if (count > 0 && (!desc || !out_pool)) return fail(LLP_E_ARG, "desc and out_pool are required");
    if (pool_words < 0 || out_words < 0) return fail(LLP_E_ARG, "pool sizes must be >= 0");
    if (pool_words > 0 && !pool) return fail(LLP_E_ARG, "pool is NULL");
    return LLP_OK;
}

static int batch_finish(hipStream_t st, BCtrl* ctrl, BCtrl* out = nullptr) {
    BCtrl h;
    int s = readback(st, ctrl, &h, sizeof(h));
    if (s) return s;
    if (out) *out = h;
    if (h.status == LLP_E_HIP) return fail(h.status, "claim order out of range");
    if (h.status == LLP_E_INPUT) return fail(h.status, "an instance is malformed or outside the pools");
    if (h.status == LLP_E_OVERFLOW) return fail(h.status, "an instance's result does not fit int32");
    if (h.status) return fail(h.status, "instance status %d", h.status);
    return LLP_OK;
}

int solve_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words, int32_t* out_pool,
                int64_t out_words, int32_t* out_status, const llp_opts* opts) {
    int s = batch_args(count, desc, pool, pool_words, out_pool, out_words);
    if (s || count == 0) return s;
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    void* ws = nullptr;
    s = batch_ws(&ws, o, count);
    if (s) return s;
    BCtrl* ctrl = (BCtrl*)ws;
    BatchPlan p;
    s = batch_plan(count, desc, o, ctrl, &p);
    if (s) return s;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    s = batch_enqueue(p, count, desc, pool, pool_words, out_pool, out_words, out_status, ctrl, st,
                      (o.flags & LLP_ASYNC) ? o.status_dev : nullptr);
    if (s) return s;
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    if (o.flags & LLP_ASYNC) return LLP_OK;
    s = batch_finish(st, ctrl);
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->candidates = count;
        if (timing) {
            float ms = 0.f;
            LLP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            o.stats->device_ms = ms;
            o.stats->kernel_ms = ms;
        }
    }
    if (timing) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    return s;
}

// ---------------------------------------------------------------- graph replay
struct GraphKey {
    const void* desc;
    const void* pool;
    const void* out_pool;
    const void* out_status;
    const void* stream;
    const void* ws;
    int count, block, chunk;
    long long pool_words, out_words;
    bool operator<(const GraphKey& o) const {
        return std::tie(desc, pool, out_pool, out_status, stream, ws, count, block, chunk, pool_words, out_words) <
               std::tie(o.desc, o.pool, o.out_pool, o.out_status, o.stream, o.ws, o.count, o.block, o.chunk,
                        o.pool_words, o.out_words);
    }
};
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    int kn_w = 0, ss_n = 0;   // largest knapsack W and SSSP n the captured launch holds
};
static std::map<GraphKey, GraphEntry> g_graphs;

static int solve_batch_graph_once(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                                  int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts,
                                  bool* outgrown);

// A replay rebuilds the limits and the claim order inside the graph; when
// the instance table at the same address now holds a larger knapsack W or
// SSSP n than the captured launch's LDS plan, the replay marks those
// instances LLP_E_INPUT and a synchronous call drops the graph, captures a
// new one and solves again.
int solve_batch_graph(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                      int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts) {
    bool outgrown = false;
    int s = solve_batch_graph_once(count, desc, pool, pool_words, out_pool, out_words, out_status, opts, &outgrown);
    if (outgrown) s = solve_batch_graph_once(count, desc, pool, pool_words, out_pool, out_words, out_status, opts,
                                             nullptr);
    return s;
}

static int solve_batch_graph_once(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                                  int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts,
                                  bool* outgrown) {
    int s = batch_args(count, desc, pool, pool_words, out_pool, out_words);
    if (s || count == 0) return s;
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    void* ws = nullptr;
    s = batch_ws(&ws, o, count);
    if (s) return s;
    BCtrl* ctrl = (BCtrl*)ws;
    int32_t* status_dev = (o.flags & LLP_ASYNC) ? o.status_dev : nullptr;
    GraphKey key{desc, pool, out_pool, out_status, o.stream, ws, count, o.block, o.chunk, pool_words, out_words};
    hipGraphExec_t exec = nullptr;
    int plan_w = 0, plan_n = 0;
    {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            exec = it->second.exec;
            plan_w = it->second.kn_w;
            plan_n = it->second.ss_n;
        }
    }
    if (!exec) {
        BatchPlan p;
        s = batch_plan(count, desc, o, ctrl, &p);
        if (s) return s;
        // capture on a private stream (the caller's may be the null stream)
        hipStream_t cs;
        LLP_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        LLP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        s = batch_enqueue(p, count, desc, pool, pool_words, out_pool, out_words, out_status, ctrl, cs, nullptr);
        hipError_t e = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        if (s) return s;
        LLP_HIP(e);
        hipGraphExec_t x = nullptr;
        LLP_HIP(hipGraphInstantiate(&x, graph, nullptr, nullptr, 0));
        std::lock_guard<std::mutex> lk(g_bmu);
        GraphEntry ge;
        ge.graph = graph;
        ge.exec = x;
        ge.device = device_info().device;
        ge.kn_w = plan_w = p.kn_w;
        ge.ss_n = plan_n = p.ss_n;
        g_graphs[key] = ge;
        exec = x;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    LLP_HIP(hipGraphLaunch(exec, st));
    if (status_dev) hipLaunchKernelGGL(k_batch_status, dim3(1), dim3(64), 0, st, ctrl, status_dev);
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    if (o.flags & LLP_ASYNC) return LLP_OK;
    BCtrl h;
    s = batch_finish(st, ctrl, &h);
    if (outgrown && (h.bad_kind || h.max_w > plan_w || h.max_n > plan_n)) {
        std::lock_guard<std::mutex> lk(g_bmu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) {
            (void)hipGraphExecDestroy(it->second.exec);
            (void)hipGraphDestroy(it->second.graph);
            g_graphs.erase(it);
        }
        *outgrown = true;
    }
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->candidates = count;
        if (timing) {
            float ms = 0.f;
            LLP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            o.stats->device_ms = ms;
            o.stats->kernel_ms = ms;
        }
    }
    if (timing) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    return s;
}

void batch_release() {
    std::lock_guard<std::mutex> lk(g_bmu);
    for (auto& kv : g_graphs) {
        (void)hipSetDevice(kv.second.device);
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
    tune_clear();
}

// ---------------------------------------------------------------- autotuner
int autotune_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                   int32_t* out_pool, int64_t out_words, char* report, size_t report_bytes, const llp_opts* opts) {
    int s = batch_args(count, desc, pool, pool_words, out_pool, out_words);
    if (s) return s;
    if (count == 0) return fail(LLP_E_ARG, "the autotuner needs a non-empty batch");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    void* ws = nullptr;
    s = batch_ws(&ws, o, count);
    if (s) return s;
    BCtrl* ctrl = (BCtrl*)ws;
    std::string rep;
    float best_ms = 1e30f;
    int best_b = 0, best_c = 0;
    hipEvent_t e0, e1;
    LLP_HIP(hipEventCreate(&e0));
    LLP_HIP(hipEventCreate(&e1));
    for (int block : {256, 512, 1024}) {
        for (int chunk : {1, 2, 4, 8}) {
            llp_opts oc = o;
            oc.block = block;
            oc.chunk = chunk;
            BatchPlan p;
            s = batch_plan(count, desc, oc, ctrl, &p);
            if (s) continue;   // this shape cannot hold the batch's largest instance
            std::vector<float> ts;
            for (int rep_i = 0; rep_i < 4 && s == LLP_OK; ++rep_i) {
                LLP_HIP(hipEventRecord(e0, st));
                s = batch_enqueue(p, count, desc, pool, pool_words, out_pool, out_words, nullptr, ctrl, st, nullptr);
                LLP_HIP(hipEventRecord(e1, st));
                LLP_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                LLP_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (rep_i > 0) ts.push_back(ms);
            }
            if (s) break;
            s = batch_finish(st, ctrl);
            if (s) break;
            std::sort(ts.begin(), ts.end());
            float med = ts[ts.size() / 2];
            char line[64];
            snprintf(line, sizeof(line), "%d %d %.4f\n", block, chunk, med);
            rep += line;
            if (med < best_ms) {
                best_ms = med;
                best_b = block;
                best_c = chunk;
            }
        }
        if (s) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    if (!best_b) return fail(LLP_E_ARG, "no launch shape can hold this batch");
    tune_record(LLP_KIND_BATCH, count, best_b, best_c);
    if (report && report_bytes) {
        size_t k = rep.size() < report_bytes - 1 ? rep.size() : report_bytes - 1;
        memcpy(report, rep.data(), k);
        report[k] = 0;
    }
    return LLP_OK;
}

int autotune_get(int kind, int32_t* block, int32_t* chunk) {
    if (kind != LLP_KIND_BATCH && kind != LLP_KIND_SSSP && kind != LLP_KIND_BFS)
        return fail(LLP_E_ARG, "only LLP_KIND_BATCH, LLP_KIND_SSSP and LLP_KIND_BFS are tuned");
    int b = 0, c = 0;
    if (!tune_last(kind, &b, &c)) return fail(LLP_E_ARG, "no tuned shape recorded on this device");
    if (block) *block = b;
    if (chunk) *chunk = c;
    return LLP_OK;
}

}  // namespace llp

extern "C" {

int llp_solve_knapsack(int32_t items, int32_t W, const int32_t* wt, const int32_t* val, int32_t* best,
                       int32_t* last_row, const llp_opts* opts) {
    return llp::solve_knapsack(items, W, wt, val, best, last_row, opts);
}

int llp_solve_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                    int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts) {
    return llp::solve_batch(count, desc, pool, pool_words, out_pool, out_words, out_status, opts);
}

int llp_solve_batch_graph(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                          int32_t* out_pool, int64_t out_words, int32_t* out_status, const llp_opts* opts) {
    return llp::solve_batch_graph(count, desc, pool, pool_words, out_pool, out_words, out_status, opts);
}

int llp_autotune_batch(int32_t count, const llp_instance* desc, const int32_t* pool, int64_t pool_words,
                       int32_t* out_pool, int64_t out_words, char* report, size_t report_bytes,
                       const llp_opts* opts) {
    return llp::autotune_batch(count, desc, pool, pool_words, out_pool, out_words, report, report_bytes, opts);
}

int llp_autotune_get(int kind, int32_t* block, int32_t* chunk) { return llp::autotune_get(kind, block, chunk); }

}  // extern "C"
