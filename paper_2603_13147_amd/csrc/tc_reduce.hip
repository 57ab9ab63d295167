// tc_reduce.hip - transitive closure (paper Section 5.7) and parallel
// reduction (Section 5.6) as LLP sweeps on gfx950.
//
// Transitive closure.  State: boolean G[u][v] packed as bit rows; (u, v) is
// forbidden while false if (u, v) is an arc or G[u][w] and G[w][v] for some
// w.  Row u is swept by one workgroup with the row and two frontier bitmaps
// in LDS: the arcs of u are set first, then every round the bits set in the
// previous round (the frontier w) set G[u][x] for each arc (w, x).  Each such
// (u, x) is forbidden in the current state (G[u][w] holds and the arc makes
// G[w][x] hold), so every advance is one of the paper's, and the row stops
// when a round sets nothing: the least fixpoint, reachability by paths of
// length >= 1.
//
// Reduction.  The tree of tiles: each workgroup sums one tile of the input
// (grid-stride, modulo 2^64) and publishes it; the root becomes forbidden once
// all its children have published, which the last workgroup to arrive at the
// counter observes, and it advances the root to the sum of the partials.
#include <string.h>

#include <map>
#include <mutex>

#include "llp_dev.h"
#include "llp_host.h"

namespace llp {

// --------------------------------------------------------------- closure
constexpr int TC_MAX_N = 65536;

struct TCtrl {
    int status;
    int pad;
    int diag[8];
    long long rounds;   // summed over rows
};

__global__ void k_tc_init(TCtrl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        TCtrl z;
        memset(&z, 0, sizeof(z));
        *c = z;
    }
}

__global__ void __launch_bounds__(256) k_tc_row(int n, int m, const int* ptr, const int* dst, unsigned* bits,
                                                TCtrl* ctl) {
    extern __shared__ unsigned tl[];
    __shared__ int any[2];
    __shared__ int bad;
    const int T = blockDim.x, t = threadIdx.x;
    const int words = (n + 31) >> 5;
    unsigned* row = tl;
    unsigned* cur = tl + words;
    unsigned* nxt = tl + 2 * words;
    const int u = blockIdx.x;
    for (int i = t; i < words; i += T) {
        row[i] = 0u;
        cur[i] = 0u;
        nxt[i] = 0u;
    }
    if (t == 0) {
        any[0] = any[1] = 0;
        bad = 0;
    }
    __syncthreads();
    // round 0: the arcs of u
    {
        int b = ptr[u], e = ptr[u + 1];
        if (b < 0 || e > m || e < b) {
            if (t == 0) bad = 1;
        } else {
            for (int k = b + t; k < e; k += T) {
                int x = dst[k];
                if ((unsigned)x >= (unsigned)n) {
                    bad = 1;
                    continue;
                }
                unsigned bit = 1u << (x & 31);
                unsigned old = atomicOr(&row[x >> 5], bit);
                if (!(old & bit)) atomicOr(&cur[x >> 5], bit);
            }
        }
    }
    __syncthreads();
    int r = 0;
    for (; r <= n && !bad; ++r) {
        bool adv = false, b2 = false;
        for (int i = t; i < words; i += T) {
            unsigned f = cur[i];
            while (f) {
                int w = (i << 5) + __ffs(f) - 1;
                f &= f - 1;
                int b = ptr[w], e = ptr[w + 1];
                if (b < 0 || e > m || e < b) {
                    b2 = true;
                    continue;
                }
                for (int k = b; k < e; ++k) {
                    int x = dst[k];
                    if ((unsigned)x >= (unsigned)n) {
                        b2 = true;
                        continue;
                    }
                    unsigned bit = 1u << (x & 31);
                    if (row[x >> 5] & bit) continue;
                    unsigned old = atomicOr(&row[x >> 5], bit);
                    if (!(old & bit)) {
                        atomicOr(&nxt[x >> 5], bit);
                        adv = true;
                    }
                }
            }
        }
        if (adv) any[r & 1] = 1;
        if (b2) bad = 1;
        __syncthreads();
        const bool more = any[r & 1] != 0 && !bad;
        for (int i = t; i < words; i += T) cur[i] = 0u;
        if (t == 0) any[(r + 1) & 1] = 0;
        __syncthreads();
        unsigned* tmp = cur;
        cur = nxt;
        nxt = tmp;
        if (!more) break;
    }
    unsigned* out = bits + (long long)u * words;
    for (int i = t; i < words; i += T) out[i] = row[i];
    if (t == 0) {
        if (bad) {
            set_status(&ctl->status, LLP_E_INPUT);
            record_diag(ctl->diag, 81, u, n, 0, 0);
        }
        atomicAdd((unsigned long long*)&ctl->rounds, (unsigned long long)(r + 1));
    }
}

size_t tc_workspace_bytes(int64_t) { return 256; }

int solve_tc(int32_t n, int64_t m, const int32_t* out_ptr, const int32_t* out_dst, uint32_t* bits,
             const llp_opts* opts) {
    if (n <= 0 || n > TC_MAX_N) return fail(LLP_E_ARG, "n must be in [1, %d] (got %d)", TC_MAX_N, n);
    if (m < 0 || m > 0x7fffffffll) return fail(LLP_E_ARG, "m out of range");
    if (!out_ptr || !bits || (m > 0 && !out_dst)) return fail(LLP_E_ARG, "out_ptr, out_dst and bits are required");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    void* ws = nullptr;
    int s = get_workspace(o, 256, &ws);
    if (s) return s;
    TCtrl* ctl = (TCtrl*)ws;
    const int words = (n + 31) / 32;
    const size_t lds = (size_t)3 * words * 4;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    hipLaunchKernelGGL(k_tc_init, dim3(1), dim3(64), 0, st, ctl);
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)k_tc_row, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
    hipLaunchKernelGGL(k_tc_row, dim3(n), dim3(256), lds, st, n, (int)m, out_ptr, out_dst, bits, ctl);
    LLP_HIP(hipGetLastError());
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    TCtrl h;
    s = readback(st, ctl, &h, sizeof(h));
    if (s) return s;
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = h.rounds;
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
    if (h.status) return fail(h.status, "malformed out-CSR (row %d: offsets or ids out of range)", h.diag[1]);
    return LLP_OK;
}

// --------------------------------------------------------------- reduction
constexpr int RB = 256;

struct RCtrl {
    unsigned int arrived;
    unsigned int pad;
};

__global__ void __launch_bounds__(RB) k_reduce(long long n, const unsigned long long* x,
                                               unsigned long long* partial, RCtrl* c, unsigned long long* result) {
    __shared__ unsigned long long ws[RB / LLP_WAVE];
    __shared__ bool last;
    unsigned long long s = 0;
    const long long stride = (long long)gridDim.x * RB * 2;
    // two independent loads in flight per thread per step
    for (long long i = (long long)blockIdx.x * RB * 2 + threadIdx.x; i < n; i += stride) {
        s += x[i];
        if (i + RB < n) s += x[i + RB];
    }
    s = (unsigned long long)wave_sum64((long long)s);
    if (lane() == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int k = 0; k < RB / LLP_WAVE; ++k) b += ws[k];
        __hip_atomic_store(&partial[blockIdx.x], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // publish the tile, then count it (release); the last arrival sees all
        unsigned prev = __hip_atomic_fetch_add(&c->arrived, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    // root: sum of the published tiles
    unsigned long long r = 0;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += RB)
        r += __hip_atomic_load(&partial[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r = (unsigned long long)wave_sum64((long long)r);
    __syncthreads();
    if (lane() == 0) ws[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int k = 0; k < RB / LLP_WAVE; ++k) b += ws[k];
        *result = b;
        c->arrived = 0u;   // ready for the next solve on this workspace
    }
}

__global__ void k_reduce_reset(RCtrl* c, int* status_dev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->arrived = 0u;
        if (status_dev) *status_dev = 0;
    }
}

static int reduce_grid(int64_t n) {
    long long g = (n + RB * 8 - 1) / (RB * 8);
    long long cap = (long long)device_info().cus * 8;
    if (g > cap) g = cap;
    return (int)(g < 1 ? 1 : g);
}

size_t reduce_workspace_bytes(int64_t) { return 256 + (size_t)2048 * 8; }

int solve_reduce(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts) {
    if (n < 0) return fail(LLP_E_ARG, "n must be >= 0");
    if (!result || (n > 0 && !x)) return fail(LLP_E_ARG, "x and result are required");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    const int grid = reduce_grid(n);
    if (grid > 2048) return fail(LLP_E_ARG, "too many tiles");
    void* ws = nullptr;
    int s = get_workspace(o, reduce_workspace_bytes(n), &ws);
    if (s) return s;
    RCtrl* c = (RCtrl*)ws;
    unsigned long long* partial = (unsigned long long*)((char*)ws + 256);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        LLP_HIP(hipEventCreate(&ev0));
        LLP_HIP(hipEventCreate(&ev1));
        LLP_HIP(hipEventRecord(ev0, st));
    }
    hipLaunchKernelGGL(k_reduce_reset, dim3(1), dim3(64), 0, st, c, (o.flags & LLP_ASYNC) ? o.status_dev : nullptr);
    hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(RB), 0, st, (long long)n, (const unsigned long long*)x, partial,
                       c, (unsigned long long*)result);
    LLP_HIP(hipGetLastError());
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    if (o.flags & LLP_ASYNC) return LLP_OK;
    LLP_HIP(hipStreamSynchronize(st));
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = 2;
        o.stats->advances = grid + 1;
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
    return LLP_OK;
}

// ---------------------------------------------------------------- no-allocation reduction
// The same reduction with its scratch (the arrival counter and one partial
// per tile) in a file-scope device array instead of a workspace: for callers
// that cannot allocate.  Each GPU holds its own copy of the array; its
// device address is looked up once per device (host code never passes the
// array's name itself to a kernel).  Calls on one GPU share the array, so
// calls that overlap on one GPU race; every call clears the counter first.
constexpr int REDUCE_MAX_TILES = 2048;
constexpr size_t REDUCE_SCRATCH_BYTES = 256 + (size_t)REDUCE_MAX_TILES * 8;
static __device__ __align__(256) unsigned char scratch[REDUCE_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch;   // device -> device address of scratch

static int scratch_ptr(void** out) {
    int dev = 0;
    LLP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void* p = nullptr;
        LLP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LLP_E_HIP, "no device address for the reduction scratch");
        it = g_scratch.emplace(dev, p).first;
    }
    *out = it->second;
    return LLP_OK;
}

int solve_reduce_noalloc(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts) {
    if (n < 0) return fail(LLP_E_ARG, "n must be >= 0");
    if (!result || (n > 0 && !x)) return fail(LLP_E_ARG, "x and result are required");
    llp_opts o = opts_or_default(opts);
    if (o.flags & LLP_TIMING) return fail(LLP_E_ARG, "LLP_TIMING is not available without allocation");
    hipStream_t st = (hipStream_t)o.stream;
    const int grid = reduce_grid(n);
    if (grid > REDUCE_MAX_TILES)
        return fail(LLP_E_ARG, "%d tiles exceed the %d partials of the static scratch", grid, REDUCE_MAX_TILES);
    void* sp = nullptr;
    int s = scratch_ptr(&sp);
    if (s) return s;
    RCtrl* c = (RCtrl*)sp;
    unsigned long long* partial = (unsigned long long*)((char*)sp + 256);
    hipLaunchKernelGGL(k_reduce_reset, dim3(1), dim3(64), 0, st, c, (o.flags & LLP_ASYNC) ? o.status_dev : nullptr);
    hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(RB), 0, st, (long long)n, (const unsigned long long*)x, partial,
                       c, (unsigned long long*)result);
    LLP_HIP(hipGetLastError());
    if (o.flags & LLP_ASYNC) return LLP_OK;
    LLP_HIP(hipStreamSynchronize(st));
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = 2;
        o.stats->advances = grid + 1;
    }
    return LLP_OK;
}

}  // namespace llp

extern "C" {

int llp_solve_reduce_noalloc(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts) {
    return llp::solve_reduce_noalloc(n, x, result, opts);
}

int llp_solve_tc(int32_t n, int64_t m, const int32_t* out_ptr, const int32_t* out_dst, uint32_t* bits,
                 const llp_opts* opts) {
    return llp::solve_tc(n, m, out_ptr, out_dst, bits, opts);
}

int llp_solve_reduce(int64_t n, const uint64_t* x, uint64_t* result, const llp_opts* opts) {
    return llp::solve_reduce(n, x, result, opts);
}

}  // extern "C"
