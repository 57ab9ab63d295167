// graph.hip - the LLP sweep for single-source shortest paths (paper Section
// 5.2) and breadth-first search (Section 5.3) on gfx950.
//
// State.  G[v] = INF - d(v) with INF = 2^31 - 1, so the bottom of the lattice
// is G = 0 (d = infinity) and every advance is an int32 atomicMax.  The
// paper's predicate "v is forbidden iff d(v) > d(u) + w(u, v) for an in-arc"
// becomes "G[v] < G[u] - w(u, v) for an in-arc with G[u] > 0", and alpha(G, v)
// is the largest such G[u] - w (Definition 3).  The source has alpha = INF.
// Any partial maximum over a subset of in-arcs is also an alpha-forbidden
// advance, which is what lets a hub's in-arcs be split across waves and the
// push rounds advance one arc at a time.
//
// Rounds.  Each round is enqueued as two kernels (PRE, MAIN); the kernel
// boundary is the grid-wide synchronisation (on gfx950 a device-side grid
// barrier, whose agent-scope fences flush and invalidate every XCD's L2 per
// wave, costs far more than a launch).  PRE reads the changed list CL[r-1],
// decides the round's mode, and either expands CL[r-1] into the candidate
// worklist WL (successor expansion, Section 4.2) or pushes along its
// out-arcs.  MAIN evaluates the candidates (or every vertex in a dense round)
// and produces CL[r].  A round whose input list is empty sets the device
// `done` flag for the host and a stop word for the next launch; later
// kernels return at once.  The host polls the flag every few rounds.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "llp_host.h"
#include "llp_lists.h"
#include "llp_sched.h"

namespace llp {

constexpr int GB = 512;            // threads per workgroup
constexpr int GW = GB / LLP_WAVE;  // waves per workgroup
constexpr int MAX_SEG = 2048;      // max workgroups per phase kernel

enum { MODE_PULL = 0, MODE_DENSE = 1, MODE_PUSH = 2 };

struct GCtrl {
    int done;
    int status;
    int last_round;
    int mode;
    int ovf;
    int verify_changed;
    int dbase;          // delta base width (2^floor(log2 mean weight), from a sample of the arcs)
    int over;           // the round limit was reached
    int decoded;        // the launch that found the end decoded G in place
    int carried[2];     // entries carried by the delta filter, by round parity (traced solves)
    int step_phase[2];  // step kernel k: phase[k & 1] 0 = PRE of round step_round + 1, 1 = MAIN of step_round
                        // (2: MAIN of a BFS dense round evaluated with the bitmap)
    int step_round[2];
    int diag[8];        // first guard event: site, index, bound, context
    long long rounds, cand, edges, adv, xedges, pedges, gath;
    long long bmr;      // BFS dense rounds evaluated with the bitmap
    SchedHist hist[2];  // scheduler history, double-buffered by round parity
    int stop[2];        // step launch k returns at once when stop[k & 1] is set (see k_graph_step)
    unsigned tail_bar;  // barrier counter of a tail launch (cleared before each)
    int tail_rounds;    // rounds run by tail launches
    int end_k;          // the step launch that found the end
};

struct GArgs {
    int n, m;
    const int* in_ptr;
    const int* in_src;
    const int* in_w;
    const int* out_ptr;
    const int* out_dst;
    const int* out_w;
    int* G;
    int* stamp;
    int* cstamp;
    ListRef wl, cl0, cl1;
    int nseg;
    int source;
    int unit_w;        // BFS: every weight is 1
    int jobs;          // job scheduling in pull form: G = S, contribution S[p] + dur[p]
    const int* vdur;   // jobs: duration per job (the weight of every out-arc of p)
    int warm_dense;    // warm start: round 1 is dense
    int fuse_end;      // the launch that finds the end decodes G (no verification, not jobs)
    GCtrl* ctrl;
    llp_trace_rec* trace;
    long long trace_cap;
    signed char* plog;     // LLP_TIMING: phase run by step launch k (-1 none, 0 PRE, 1 MAIN)
    long long plog_cap;
    long long max_rounds;
    SchedParams sp;
    int dbase_known;       // > 0: the delta base width of these weights, sampled by an earlier solve
    unsigned long long* bm;   // BFS dense rounds: bit v set iff d(v) <= dmin of the round (n bits)
};

__device__ __forceinline__ ListRef cl_of(const GArgs& a, int r) { return (r & 1) ? a.cl1 : a.cl0; }

// --------------------------------------------------------------- init
// Workgroup 0 writes the control block, the list words and CL[0], after its
// sample of the arcs' weights (a chain of random loads); the other workgroups
// clear the state meanwhile, so the sample is off the launch's critical path.
// A launch of one workgroup does both.
__global__ void k_graph_init(GArgs a, const int* warm) {
    const bool clears = gridDim.x == 1 || blockIdx.x > 0;
    const long long nb = gridDim.x > 1 ? gridDim.x - 1 : 1;
    const long long tid = (gridDim.x > 1 ? blockIdx.x - 1 : 0) * (long long)blockDim.x + threadIdx.x;
    const long long nt = nb * blockDim.x;
    for (long long v = tid; clears && v < a.n; v += nt) {
        int g = 0;
        if (a.jobs) {
            g = warm && warm[v] > 0 ? warm[v] : 0;
        } else {
            if (warm) {
                int d = warm[v];
                g = (d >= LLP_INF || d < 0) ? 0 : LLP_INF - d;
            }
            if (v == a.source) g = LLP_INF;
        }
        a.G[v] = g;
        a.stamp[v] = 0;
        a.cstamp[v] = 0;
    }
    if (blockIdx.x == 0) {
        // the list words (segment 0's is seeded below, after the barrier)
        for (int s = threadIdx.x; s < a.nseg; s += blockDim.x) {
            a.cl0.seg[s] = 0ull;
            a.cl1.seg[s] = 0ull;
            a.wl.seg[s] = 0ull;
            a.cl0.segmin[s] = LLP_INF;
            a.cl1.segmin[s] = LLP_INF;
        }
        // delta base width: 2^floor(log2 of the mean weight of a stride sample of
        // the in-arcs) (1 for unit weights)
        __shared__ long long wsum[4];
        long long sum = 0;
        int cnt = 0;
        if (!a.unit_w && !a.jobs && a.in_w && a.m > 0 && a.dbase_known <= 0) {
            // sample i of 4096 is arc i m / 4096; the 16 loads of a thread
            // are issued before any is summed (the launch has 256 threads)
            int wv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = threadIdx.x + q * 256;
                wv[q] = (threadIdx.x < 256) ? a.in_w[((long long)i * a.m) >> 12] : 0;
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) sum += wv[q];
            cnt = 4096;
        }
        sum = wave_sum64(sum);
        if (lane() == 0) wsum[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long t = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wsum[k];
            int base = a.dbase_known > 0 ? a.dbase_known : 1;
            if (cnt) {
                long long mean = t / cnt;
                while ((long long)base * 2 <= mean && base < (1 << 29)) base *= 2;
            }
            GCtrl c;
            memset(&c, 0, sizeof(c));
            c.mode = -1;
            c.dbase = base;
            *a.ctrl = c;
            if (!a.jobs) {
                // CL[0] = {source}: one entry in segment 0, distance 0
                int ob = a.out_ptr ? a.out_ptr[a.source] : 0;
                int od = a.out_ptr ? a.out_ptr[a.source + 1] - ob : 0;
                if (od > 0) {
                    a.cl0.ent[0] = make_int4(a.source, ob, 0, od);
                    a.cl0.seg[0] = 1ull | ((unsigned long long)(unsigned)od << 32);
                    a.cl0.segmin[0] = 0;
                }
            }
        }
    }
}

// --------------------------------------------------------------- validation
__global__ void k_graph_validate(GArgs a) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    int bad = 0;
    for (long long v = tid; v <= a.n; v += nt) {
        int p = a.in_ptr[v];
        if (v == 0 && p != 0) bad = 1;
        if (v == a.n && p != a.m) bad = 1;
        if (v < a.n && a.in_ptr[v + 1] < p) bad = 1;
        if (v < a.n && a.jobs && a.vdur[v] < 0) bad = 1;
        if (a.out_ptr) {
            int q = a.out_ptr[v];
            if (v == 0 && q != 0) bad = 1;
            if (v == a.n && q != a.m) bad = 1;
            if (v < a.n && a.out_ptr[v + 1] < q) bad = 1;
        }
    }
    for (long long e = tid; e < a.m; e += nt) {
        int u = a.in_src[e];
        if (u < 0 || u >= a.n) bad = 1;
        if (!a.unit_w && a.in_w && a.in_w[e] < 0) bad = 1;
        if (a.out_dst) {
            int x = a.out_dst[e];
            if (x < 0 || x >= a.n) bad = 1;
        }
        if (!a.unit_w && a.out_w && a.out_w[e] < 0) bad = 1;
    }
    if (bad) set_status(&a.ctrl->status, LLP_E_INPUT);
}

// --------------------------------------------------------------- helpers
// Dense rounds evaluate rows in blocks of at most DBLK arcs (every row of up
// to DBLK in-arcs lies in one block; a row of at most DSHORT arcs is reduced
// by one lane, a longer one by the whole wave), rows of up to DLONG in-arcs
// are evaluated by one wave, longer rows are split between waves by arc range.
constexpr int DBLK = 512;     // arcs per block: 8 per lane
constexpr int DSHORT = 64;    // longest row reduced by a single lane
constexpr int DLONG = 1024;   // longest row evaluated by a single wave

struct GShared {
    int cnt[MAX_SEG];
    int epre[MAX_SEG + 1];
    union {
        int own[GW][64];      // list iterator: owner slots
        int dcb[GW][DBLK + 192];  // dense blocks: candidate (or row) of each position; per row: bound, first arc, first position
        struct {
            int pw[GW][8][64];    // push blocks: entry start, source value, row base, duration; entry of each position
            int lq_v[512], lq_ob[512], lq_od[512];   // bucketed push rounds: the local queue (see local_drain)
        };
    };
    unsigned long long ctr;    // appends to the phase's main output list
    unsigned long long cctr;   // PRE in pull rounds: entries carried into CL[r]
    int cmin;                  // smallest distance appended to CL[r] by this workgroup
    int tot_edges, tot_count;
    int code;
    int tmp1;
    int carried;
    int tmp[GW + 1];
    int lq_top;                // entries of the local queue
    long long lq_arcs;         // arcs the local passes pushed
    unsigned long long cnt_rd, cnt_gath;   // dense rounds: arcs read, states gathered by the workgroup
};

// Candidate value pulled through arc (u -> v) of weight w: G[u] - w when u is
// reached and the result stays a reached value; flags overflow otherwise.
__device__ __forceinline__ int pull_cand(int gu, int w, bool& ovf) {
    if (gu <= 0) return 0;
    int c = gu - w;
    if (c <= 0) { ovf = true; return 0; }
    return c;
}

// Jobs: start time published through arc (p -> j) is S[p] + dur[p]; a sum
// beyond int32 means p's completion time overflows.
__device__ __forceinline__ int jobs_cand(int sp, int dp, bool& ovf) {
    long long c = (long long)sp + dp;
    if (c > LLP_INF) { ovf = true; return LLP_INF; }
    return (int)c;
}

// Distance key of a changed vertex for the delta buckets (its decoded
// distance; jobs have no buckets and use 0).
__device__ __forceinline__ int dist_key(const GArgs& a, int g) { return a.jobs ? 0 : LLP_INF - g; }

// Evaluate edges of the iteration: segmented max of candidates per owner,
// advance owners by atomicMax, append changed vertices to CL.
__device__ __forceinline__ void eval_body(const GArgs& a, const EdgeCtx& c, int r, const ListRef& out,
                                          GShared& sh, bool& ovf, long long& nadv) {
    const int l = lane();
    // the segment structure is known before any gather: the tail lane of each
    // owner's run reads the owner's state while the arcs' sources are gathered
    int seg = c.active ? c.j : 64 + l;
    int nseg = __shfl_down(seg, 1, LLP_WAVE);
    bool tail = c.active && (l == 63 || nseg != seg);
    int v = guard(c.own.x, a.n, a.ctrl->diag, 43, c.j, c.own.z);
    int gv = tail ? a.G[v] : 0;
    int cand = 0;
    if (c.active) {
        int e = guard(c.csr, a.m, a.ctrl->diag, 41, c.own.y, c.own.z);
        int u = guard(a.in_src[e], a.n, a.ctrl->diag, 42, e, 0);
        if (a.jobs) {
            cand = jobs_cand(a.G[u], a.vdur[u], ovf);
        } else {
            int w = a.unit_w ? 1 : a.in_w[e];
            cand = pull_cand(a.G[u], w, ovf);
        }
    }
    int x = seg_incl_max(cand, seg);
    bool changed = false, advanced = false;
    int ob = 0, od = 0;
    if (tail && x > 0 && x > gv) {
        int old = amax(&a.G[v], x);
        advanced = old < x;
        if (advanced) {
            // the row offsets do not depend on the stamp: load them alongside
            ob = a.out_ptr[v];
            int oe = a.out_ptr[v + 1];
            changed = (amax(&a.cstamp[v], r) < r);
            od = oe - ob;
        }
    }
    if (changed) nadv++;
    append(changed && od > 0, v, ob, od, &sh.ctr, out, &a.ctrl->status);
    // every advanced vertex is in CL[r] (appended now, earlier this round, or
    // carried), so its new distance bounds the list's minimum
    if (out.segmin) wave_min_to_lds(advanced, dist_key(a, x), &sh.cmin);
}

// Candidates of N in-arcs with sources u[] (valid indices) and weights w[]:
// all gathers are issued before any result is used; inactive arcs (act
// false) give 0.
template <int N>
__device__ __forceinline__ void arc_cands(const GArgs& a, const int* u, const int* w, const bool* act, int* c,
                                          bool& ovf) {
    int gu[N];
#pragma unroll
    for (int j = 0; j < N; ++j) gu[j] = a.G[u[j]];
    if (a.jobs) {
        int du[N];
#pragma unroll
        for (int j = 0; j < N; ++j) du[j] = a.vdur[u[j]];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            bool o = false;
            const int x = jobs_cand(gu[j], du[j], o);
            c[j] = act[j] ? x : 0;
            ovf |= act[j] && o;
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            bool o = false;
            const int x = pull_cand(gu[j], w[j], o);
            c[j] = act[j] ? x : 0;
            ovf |= act[j] && o;
        }
    }
}

// BFS dense round with the bitmap: an arc from a marked tail (distance at
// most dmin) offers its row exactly the cap INF - (dmin + 1); other arcs
// offer nothing this round (their tails are carried, see pre_phase).
template <int N>
__device__ __forceinline__ void arc_cands_bm(const GArgs& a, const int* u, const bool* act, int* c, int cap) {
    unsigned long long b[N];
#pragma unroll
    for (int j = 0; j < N; ++j) b[j] = a.bm[u[j] >> 6];
#pragma unroll
    for (int j = 0; j < N; ++j) c[j] = (act[j] && ((b[j] >> (u[j] & 63)) & 1ull)) ? cap : 0;
}

// State of rows v .. v+63, one per lane: in-row bounds, value, out-row bounds.
struct RowWin {
    int pl, pn, g, ob, oe;
};

__device__ __forceinline__ RowWin load_rows(const GArgs& a, int v) {
    RowWin w{0, 0, 0, 0, 0};
    const int x = v + lane();
    if (x < a.n) {
        w.pl = a.in_ptr[x];
        w.pn = a.in_ptr[x + 1];
        w.g = a.G[x];
        w.ob = a.out_ptr[x];
        w.oe = a.out_ptr[x + 1];
    }
    return w;
}

// Arc bound of a row with state g in a dense round of a weighted graph: an
// arc of weight w can improve the row only if w < d - dlo, d = LLP_INF - g
// its current distance and dlo the smallest distance in CL[r-1] (see
// dense_dmin).  No bound (INT_MAX) without dlo or for an unreached row.
__device__ __forceinline__ int arc_bound(int g, int dlo) {
    if (dlo < 0 || g <= 0) return 0x7fffffff;
    return (LLP_INF - g) - dlo;
}

// Advance index v to x if it improves on gv (lane 0's values).  whole: this
// wave saw every in-arc of v in this phase and is its only writer, so the
// value is stored and v appended directly; otherwise atomicMax, and the stamp
// decides which advancing wave appends v.
__device__ __forceinline__ void row_advance(const GArgs& a, int r, int v, int x, int gv, int ob, int oe, bool whole,
                                            const ListRef& out, GShared& sh, long long& nadv, int& lmin) {
    bool changed = false, advanced = false;
    if (lane() == 0 && x > 0 && x > gv) {
        if (whole) {
            __hip_atomic_store(&a.G[v], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            advanced = changed = true;
        } else {
            advanced = amax(&a.G[v], x) < x;
            if (advanced) changed = amax(&a.cstamp[v], r) < r;
        }
    }
    if (changed) nadv++;
    if (advanced) lmin = min(lmin, dist_key(a, x));
    append(changed && oe > ob, v, ob, oe - ob, &sh.ctr, out, &a.ctrl->status);
}

// Wave-wide evaluation of in-arcs [lo, hi) of row v (8 arcs per lane per
// iteration); returns the maximum candidate in every lane.
// cap: no candidate can exceed it (see dense_cap), so the scan stops once
// one reaches it; gv_live: re-read the row's state before each chunk (the
// row is split between waves, another may already have reached the cap).
// thr: only arcs of weight below it can improve the row (see dense_dmin);
// the others are not gathered.  nrd: arcs read, nins: states gathered.
template <bool BM>
__device__ __forceinline__ int row_max(const GArgs& a, int lo, int hi, bool& ovf, int cap, int v, bool gv_live,
                                       int thr, int& nrd, int& nins) {
    const int l = lane();
    constexpr bool look = BM;
    const bool weighted = !a.unit_w && !a.jobs;
    int x = 0;
    bool bad = false;
    for (int b = lo; b < hi; b += DBLK) {
        if (b > lo && __any(x >= cap)) break;
        if (gv_live && cap < LLP_INF && ld_relaxed(&a.G[v]) >= cap) break;
        // every load of the chunk is issued before any loaded index is checked
        int u[8], w[8], c[8];
        bool act[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int i = b + l + 64 * j;
            act[j] = i < hi;
            const int e = act[j] ? clampi(i, a.m, bad) : 0;
            u[j] = act[j] ? __builtin_nontemporal_load(a.in_src + e) : 0;
            w[j] = (act[j] && weighted) ? __builtin_nontemporal_load(a.in_w + e) : 1;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            nrd += act[j] ? 1 : 0;
            if (act[j] && w[j] >= thr) {
                act[j] = false;
                u[j] = 0;
            }
            if constexpr (!look) nins += act[j] ? 1 : 0;   // bitmap lookups gather no state
            u[j] = clampi(u[j], a.n, bad);
        }
        if constexpr (look) arc_cands_bm<8>(a, u, act, c, cap);
        else arc_cands<8>(a, u, w, act, c, ovf);
#pragma unroll
        for (int j = 0; j < 8; ++j) x = max(x, c[j]);
    }
    if (bad) record_diag(a.ctrl->diag, 44, lo, hi, a.m, a.n);
    return wave_max(x);
}

// Dense evaluation of one wave's arc range [wb, we): every row whose first
// in-arc lies in the range (rows of up to DLONG arcs are evaluated whole,
// even past we) and the part inside the range of any longer row.  BM: a BFS
// round whose tails are looked up in the bitmap instead of gathered.
template <bool BM>
__device__ void dense_wave(const GArgs& a, int r, int wb, int we, const ListRef& out, GShared& sh, int* cb,
                           bool& ovf, long long& nadv, int& lmin, int cap, int dlo, int& nrd, int& nins) {
    if (wb >= we) return;
    const int l = lane();
    constexpr bool look = BM;
    DenseSrc ds{a.in_ptr, a.n, a.ctrl->diag};
    int v = ds.locate(wb).s;
    RowWin R = load_rows(a, v);
    bool first = true;
    while (v < a.n) {
        const int P0 = shfl(R.pl, 0), P1 = shfl(R.pn, 0);
        if (P0 >= we) break;
        const int d0 = P1 - P0;
        if (first && P0 < wb) {
            // row v starts in an earlier wave's range: only a long row has a part here
            first = false;
            const RowWin Rn = load_rows(a, v + 1);
            if (d0 > DLONG) {
                const int g0 = shfl(R.g, 0);
                const int x = g0 >= cap ? 0 : row_max<BM>(a, wb, min(we, P1), ovf, cap, v, true, arc_bound(g0, dlo), nrd, nins);
                row_advance(a, r, v, x, shfl(R.g, 0), shfl(R.ob, 0), shfl(R.oe, 0), false, out, sh, nadv, lmin);
            }
            R = Rn;
            ++v;
            continue;
        }
        first = false;
        // a row at the bound is final (see dense_cap): none of its arcs is read
        if (d0 > DBLK && !(cap < LLP_INF && shfl(R.g, 0) >= cap)) {
            const RowWin Rn = load_rows(a, v + 1);
            const int hi = d0 <= DLONG ? P1 : min(we, P1);
            const int g0 = shfl(R.g, 0);
            const int x = g0 >= cap ? 0 : row_max<BM>(a, P0, hi, ovf, cap, v, hi != P1, arc_bound(g0, dlo), nrd, nins);
            row_advance(a, r, v, x, shfl(R.g, 0), shfl(R.ob, 0), shfl(R.oe, 0), hi == P1, out, sh, nadv, lmin);
            R = Rn;
            ++v;
            continue;
        }
        // a block of rows v .. v+k-1, all starting inside the range, whose
        // arcs to read number at most DBLK: a final row has none, so the
        // block's positions 0 .. C-1 run over the other rows' arcs in order
        // (row l from position cs)
        const bool finl = cap < LLP_INF && v + l < a.n && R.g >= cap;
        const int len = (v + l < a.n && !finl) ? R.pn - R.pl : 0;
        const int incl = cap < LLP_INF ? wave_incl_sum(len) : R.pn - P0;   // no final rows: arcs in order
        const bool ok = v + l < a.n && R.pl < we && incl <= DBLK;
        const uint64_t stop = ~ballot(ok);
        const int k = stop ? __ffsll((long long)stop) - 1 : 64;   // >= 1: row v qualifies
        const int C = shfl(incl, k - 1);
        const int cs = incl - len;
        const RowWin Rn = load_rows(a, v + k);
        const uint64_t fin = ballot(l < k && finl);
        // weighted graphs: each row's arc bound (see dense_dmin), when any
        // row of the block has one
        const int thr = l < k ? arc_bound(R.g, dlo) : 0x7fffffff;
        const bool lim = ballot(thr != 0x7fffffff) != 0ull;
        // the row of each arc position, when some row of the block is final
        // (positions skip its arcs) or has a bound: row l writes l at its
        // first position over a fill of -1, and a max-scan over the positions
        // fills the rest (position 0 starts the first row with arcs; cb
        // holds this table until the candidates are written); per row: rt its
        // arc bound, ra its first arc, rc its first position
        int* rt = cb + DBLK;
        int* ra = rt + 64;
        int* rc = ra + 64;
        const bool table = fin || lim;
        if (table) {
            rt[l] = thr;
            if (fin) {
                ra[l] = R.pl;
                rc[l] = cs;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) cb[8 * l + j] = -1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (l < k && len > 0) cb[cs] = l;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int q[8], run = -1;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                run = max(run, cb[8 * l + j]);
                q[j] = run;
            }
            int before = __shfl_up(wave_incl_max(run), 1, LLP_WAVE);
            if (l == 0) before = -1;
#pragma unroll
            for (int j = 0; j < 8; ++j) cb[8 * l + j] = max(before, q[j]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // every load of the block is issued before any loaded index is checked
        const bool weighted = !a.unit_w && !a.jobs;
        bool bad = false;
        int u[8], w[8], c[8], t[8];
        bool act[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int p = l + 64 * j;
            act[j] = p < C;
            t[j] = 0x7fffffff;
            int i = P0 + p;
            if (table && act[j]) {
                const int o = cb[p];
                t[j] = rt[o];
                if (fin) i = ra[o] + (p - rc[o]);   // positions skip the final rows' arcs
            }
            const int e = act[j] ? clampi(i, a.m, bad) : 0;
            u[j] = act[j] ? __builtin_nontemporal_load(a.in_src + e) : 0;
            w[j] = (act[j] && weighted) ? __builtin_nontemporal_load(a.in_w + e) : 1;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            nrd += act[j] ? 1 : 0;
            if (act[j] && w[j] >= t[j]) {   // cannot improve its row: no gather
                act[j] = false;
                u[j] = 0;
            }
            if constexpr (!look) nins += act[j] ? 1 : 0;
            u[j] = clampi(u[j], a.n, bad);
        }
        if constexpr (look) arc_cands_bm<8>(a, u, act, c, cap);
        else arc_cands<8>(a, u, w, act, c, ovf);
#pragma unroll
        for (int j = 0; j < 8; ++j) cb[l + 64 * j] = c[j];   // positions past the block are never read
        if (bad) record_diag(a.ctrl->diag, 46, v, P0, C, a.n);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int x = 0;
        const int lo = cs, hi = cs + len;   // positions of the row: within [0, DBLK]
        if (l < k && hi - lo <= DSHORT) {
            // four independent maxima: four LDS reads in flight
            int i = lo, x1 = 0, x2 = 0, x3 = 0;
            for (; i + 4 <= hi; i += 4) {
                x = max(x, cb[i]);
                x1 = max(x1, cb[i + 1]);
                x2 = max(x2, cb[i + 2]);
                x3 = max(x3, cb[i + 3]);
            }
            for (; i < hi; ++i) x = max(x, cb[i]);
            x = max(max(x, x1), max(x2, x3));
        }
        // the block's longer rows (at most DBLK / DSHORT of them): whole wave
        for (uint64_t big = ballot(l < k && hi - lo > DSHORT); big; big &= big - 1) {
            const int rl = __ffsll((long long)big) - 1;
            const int s = shfl(lo, rl), e = shfl(hi, rl);
            int y = 0;
            for (int i = s + l; i < e; i += 64) y = max(y, cb[i]);
            y = wave_max(y);
            if (l == rl) x = y;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const bool adv = l < k && x > 0 && x > R.g;
        if (adv) {
            __hip_atomic_store(&a.G[v + l], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            nadv++;
            lmin = min(lmin, dist_key(a, x));
        }
        append(adv && R.oe > R.ob, v + l, R.ob, R.oe - R.ob, &sh.ctr, out, &a.ctrl->status);
        R = Rn;
        v += k;
    }
}

// Push over virtual edges [wb, we) of a changed list, PBLK arcs per block:
// a block covers at most 64 entries, each lane pushes PJ arcs of it (single-
// arc partial advances, Definition 3).  An arc finds its entry by binary
// search over the block's entry starts in LDS.  Delta buckets: an entry at
// distance >= hi is carried into CL[r] (by the block where it starts) and
// none of its arcs is pushed; the test is monotone (distances only fall), so
// an entry pushed in part is never carried.
constexpr int PJ = 2;
constexpr int PBLK = 64 * PJ;

// Local queue of a bucketed push round (the per-worker work bag of the
// paper's Section 4.3 with its recency preference, per workgroup): a target
// the workgroup advances to a distance inside the round's bucket, with at
// most LQ_DEG out-arcs, goes onto a stack in LDS instead of into CL[r], and
// after its share of the list the workgroup pops the newest entries and
// pushes their arcs with their current values, queueing again what those
// advance, for at most LQ_ITERS passes.  What does not fit, and what is left
// after the last pass, is stamped and appended to CL[r] as usual, so every
// advanced vertex has its arcs pushed with its final value either here or in
// a later round.  The bucket bounds how far a pass can run ahead.
constexpr int LQ_CAP = 512;
constexpr int LQ_DEG = 8;
constexpr int LQ_ITERS = 64;

// Queue target x (out-row [ob, ob + od)) if it qualifies and there is room;
// returns whether it was queued.
__device__ __forceinline__ bool lq_put(GShared& sh, bool want, int x, int ob, int od) {
    if (!want) return false;
    const int slot = atomicAdd(&sh.lq_top, 1);
    if (slot >= LQ_CAP) return false;
    sh.lq_v[slot] = x;
    sh.lq_ob[slot] = ob;
    sh.lq_od[slot] = od;
    return true;
}

// In-round continuation (push rounds): a lane that advanced a target with at
// most CDEG out-arcs pushes that target's arcs right away with its new
// value, up to CDEPTH steps deep, instead of leaving it to the next round;
// targets it does not continue through are stamped and appended as usual.
// A continued vertex is not stamped, so if it advances again later in the
// round its advancer appends it.  Chains (vertices of one or two out-arcs)
// are what it shortens; through wider fan-out (a weighted mesh) it spreads
// values that later rounds must correct, so it stops there.  In a round with
// delta buckets it continues only through targets whose new distance lies
// below the bucket's ceiling, as the round would have pushed them.
constexpr int CDEG = 2;
constexpr int CDEPTH = 32;
constexpr int CONT_EDGES = 1 << 22;   // rounds with at most this many arcs to push

template <bool COH>
__device__ void push_continue(const GArgs& a, int r, int cv, int cg, int cob, int cod, long long hi, const ListRef& out,
                              unsigned long long* ctr, bool& ovf, long long& nadv, int& lmin) {
    for (int d = 0; d < CDEPTH; ++d) {
        if (!__any(cv >= 0)) return;
        int y[CDEG], cand[CDEG], gy[CDEG];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < CDEG; ++k) {
            const bool act = cv >= 0 && k < cod;
            const int e = act ? clampi(cob + k, a.m, bad) : 0;
            y[k] = a.out_dst[e];
            const int w = a.unit_w ? 1 : a.out_w[e];
            bool o = false;
            const int cc = pull_cand(cg, w, o);
            ovf |= act && o;
            cand[k] = act ? cc : 0;
        }
#pragma unroll
        for (int k = 0; k < CDEG; ++k) y[k] = clampi(y[k], a.n, bad);
#pragma unroll
        for (int k = 0; k < CDEG; ++k) gy[k] = a.G[y[k]];
        if (bad) record_diag(a.ctrl->diag, 64, cv, cob, cod, a.n);
        int nv = -1, ng = 0, nob = 0, nod = 0;
#pragma unroll
        for (int k = 0; k < CDEG; ++k) {
            bool changed = false;
            int yob = 0, yod = 0;
            if (cand[k] > 0 && cand[k] > gy[k] && amax(&a.G[y[k]], cand[k]) < cand[k]) {
                yob = a.out_ptr[y[k]];
                yod = a.out_ptr[y[k] + 1] - yob;
                lmin = min(lmin, dist_key(a, cand[k]));
                if (nv < 0 && yod > 0 && yod <= CDEG && d + 1 < CDEPTH &&
                    (hi <= 0 || (long long)(LLP_INF - cand[k]) < hi)) {
                    nv = y[k];
                    ng = cand[k];
                    nob = yob;
                    nod = yod;
                } else {
                    changed = amax(&a.cstamp[y[k]], r) < r;
                }
            }
            if (changed) nadv++;
            append<COH>(changed && yod > 0, y[k], yob, yod, ctr, out, &a.ctrl->status);
        }
        cv = nv;
        cg = ng;
        cob = nob;
        cod = nod;
    }
}

template <bool COH, bool LQ, class Src>
__device__ void push_wave(const GArgs& a, const Src& src, int wb, int we, int r, long long hi, const ListRef& out,
                          unsigned long long* ctr, GShared& sh, int (*pw)[64], bool& ovf, long long& nadv,
                          int& lmin) {
    if (wb >= we) return;
    const int l = lane();
    const bool lq = LQ && hi > 0 && !a.jobs;   // bucketed rounds queue locally instead of continuing
    const bool cont = !lq && !a.jobs && src.sv.total_edges <= CONT_EDGES;
    Cursor cur = src.locate(wb);
    int base = wb;
    int av = src.avail(cur);
    int4 e = (l < av) ? src.load(cur, l) : make_int4(0, 0, LLP_INF, 0);
    while (base < we) {
        if (av <= 0) {
            if (l == 0) record_diag(a.ctrl->diag, 32, base, we, cur.s, cur.i);
            return;
        }
        const bool valid = l < av;
        const int nv = av < 64 ? av : 64;
        const int end_last = shfl(e.z + e.w, nv - 1);
        const int limit = min(min(base + PBLK, we), end_last);
        if (limit <= base) {              // inconsistent list: record and stop this wave
            if (l == 0) record_diag(a.ctrl->diag, 33, base, end_last, cur.s, cur.i);
            return;
        }
        const int done = __popcll(ballot(valid && e.z + e.w <= limit));
        const Cursor nxt = src.advance(cur, done);
        int nav = 0;
        int4 ne = make_int4(0, 0, LLP_INF, 0);
        if (limit < we) {
            nav = src.avail(nxt);
            if (l < nav) ne = src.load(nxt, l);
        }
        // the block's entries: value, carry decision, LDS tables
        int u = 0, gu = 0, du = 0;
        bool carry = false;
        if (valid) {
            u = guard(e.x, a.n, a.ctrl->diag, 61);
            gu = ld_relaxed(&a.G[u]);
            if (a.jobs) du = a.vdur[u];
            carry = hi > 0 && (long long)(LLP_INF - gu) >= hi;
        }
        const bool put = carry && e.z >= base && e.z < limit;
        if (put) amax(&a.cstamp[u], r);
        append<COH>(put, e.x, e.y, e.w, ctr, out, &a.ctrl->status);
        if (put) lmin = min(lmin, LLP_INF - gu);
        const int kc = __popcll(ballot(put));
        if (l == 0 && kc && a.trace) atomicAdd(&sh.carried, kc);
        pw[1][l] = carry ? 0 : gu;
        pw[2][l] = e.y - e.z;
        pw[3][l] = du;
        // entry of each of the block's positions: every entry starting in
        // the block (entry 0 may start before it) writes l + 1 at its first
        // position and a max-scan over the positions fills the rest
        int* tab = &pw[4][0];
#pragma unroll
        for (int j = 0; j < 4; ++j) tab[4 * l + j] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid && e.z < limit) tab[e.z > base ? e.z - base : 0] = l + 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        {
            int q[4], run = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                run = max(run, tab[4 * l + j]);
                q[j] = run;
            }
            int before = __shfl_up(wave_incl_max(run), 1, LLP_WAVE);
            if (l == 0) before = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) tab[4 * l + j] = max(before, q[j]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // arcs: entry from the table, then every load before any check
        int x[PJ], c[PJ], g[PJ], d[PJ], w[PJ];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
            const int p = base + l + 64 * j;
            g[j] = 0;
            d[j] = 0;
            int ei = 0;
            if (p < limit) {
                const int o = tab[l + 64 * j] - 1;   // last entry starting at or before p
                g[j] = pw[1][o];
                d[j] = pw[3][o];
                ei = clampi(p + pw[2][o], a.m, bad);
            }
            x[j] = a.out_dst[ei];                          // inactive arcs read position 0
            w[j] = (!a.unit_w && !a.jobs) ? a.out_w[ei] : 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
            x[j] = clampi(x[j], a.n, bad);
            c[j] = g[j] <= 0 ? 0 : (a.jobs ? jobs_cand(g[j], d[j], ovf) : pull_cand(g[j], w[j], ovf));
        }
        if (bad) record_diag(a.ctrl->diag, 62, base, limit, nv, a.n);
        int gx[PJ];
#pragma unroll
        for (int j = 0; j < PJ; ++j) gx[j] = a.G[x[j]];
#pragma unroll
        for (int j = 0; j < PJ; ++j) gx[j] = c[j] > 0 ? gx[j] : LLP_INF;
        int cv = -1, cg = 0, cob = 0, cod = 0;   // this lane's continuation
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
            bool changed = false;
            int ob = 0, od = 0;
            if (c[j] > gx[j]) {
                const int old = amax(&a.G[x[j]], c[j]);
                if (old < c[j]) {
                    ob = a.out_ptr[x[j]];
                    od = a.out_ptr[x[j] + 1] - ob;
                    const bool inb = (long long)(LLP_INF - c[j]) < hi;
                    if (LQ && lq_put(sh, lq && inb && od > 0 && od <= LQ_DEG, x[j], ob, od)) {
                        // queued: its arcs are pushed by this workgroup's local passes
                    } else if (cont && cv < 0 && od > 0 && od <= CDEG && (hi <= 0 || inb)) {
                        lmin = min(lmin, dist_key(a, c[j]));
                        cv = x[j];
                        cg = c[j];
                        cob = ob;
                        cod = od;
                    } else {
                        lmin = min(lmin, dist_key(a, c[j]));
                        changed = amax(&a.cstamp[x[j]], r) < r;
                    }
                }
            }
            if (changed) nadv++;
            append<COH>(changed && od > 0, x[j], ob, od, ctr, out, &a.ctrl->status);
        }
        if (cont) push_continue<COH>(a, r, cv, cg, cob, cod, hi, out, ctr, ovf, nadv, lmin);
        cur = nxt;
        base = limit;
        av = nav;
        e = ne;
    }
}

// The local passes of a bucketed push round (see LQ_CAP): called by every
// thread of the workgroup after its share of the list.  Each pass takes up
// to GB of the newest entries, one per thread, and pushes the entry's
// out-arcs (at most LQ_DEG) with the vertex's current value.
template <bool COH>
__device__ void local_drain(const GArgs& a, int r, long long hi, const ListRef& out, unsigned long long* ctr,
                            GShared& sh, bool& ovf, long long& nadv, int& lmin) {
    long long arcs = 0;
    for (int it = 0;; ++it) {
        __syncthreads();
        const int top = min(sh.lq_top, LQ_CAP);
        if (top == 0) break;
        // every queued entry may still have to be appended, and a pass can add
        // LQ_DEG - 1 entries per entry it takes: passes run while the
        // workgroup's segment of CL[r] can hold that, else the queue is handed
        // to the list
        const long long room = (long long)out.cap - (long long)(sh.ctr & 0xffffffffull) - top;
        int take = min(top, GB);
        if ((long long)take * (LQ_DEG - 1) > room) take = (int)max(room / (LQ_DEG - 1), 0ll);
        const bool last = it >= LQ_ITERS || take == 0;
        if (last) take = top;
        const int base = top - take;
        // the thread's entries, read before the stack is shortened and refilled
        int v[2] = {-1, -1}, ob[2] = {0, 0}, od[2] = {0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = base + threadIdx.x + q * GB;
            if (i < top) {
                v[q] = sh.lq_v[i];
                ob[q] = sh.lq_ob[i];
                od[q] = sh.lq_od[i];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) sh.lq_top = base;
        __syncthreads();
        if (last) {
            // hand what is left to the next round
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                bool changed = false;
                if (v[q] >= 0) {
                    changed = amax(&a.cstamp[v[q]], r) < r;
                    lmin = min(lmin, dist_key(a, ld_relaxed(&a.G[v[q]])));
                }
                if (changed) nadv++;
                append<COH>(changed, v[q], ob[q], od[q], ctr, out, &a.ctrl->status);
            }
            break;
        }
        const int gv = v[0] >= 0 ? ld_relaxed(&a.G[v[0]]) : 0;
        bool bad = false;
        int x[LQ_DEG], cand[LQ_DEG];
#pragma unroll
        for (int k = 0; k < LQ_DEG; ++k) {
            const bool act = v[0] >= 0 && k < od[0];
            const int e = act ? clampi(ob[0] + k, a.m, bad) : 0;
            x[k] = act ? a.out_dst[e] : 0;
            const int w = act ? (a.unit_w ? 1 : a.out_w[e]) : 0;
            bool o = false;
            const int cc = act ? pull_cand(gv, w, o) : 0;
            ovf |= act && o;
            cand[k] = cc;
            arcs += act ? 1 : 0;
        }
        int gx[LQ_DEG];
#pragma unroll
        for (int k = 0; k < LQ_DEG; ++k) {
            x[k] = clampi(x[k], a.n, bad);
            gx[k] = a.G[x[k]];
        }
        if (bad) record_diag(a.ctrl->diag, 67, v[0], ob[0], od[0], a.n);
#pragma unroll
        for (int k = 0; k < LQ_DEG; ++k) {
            bool changed = false;
            int yob = 0, yod = 0;
            if (cand[k] > 0 && cand[k] > gx[k] && amax(&a.G[x[k]], cand[k]) < cand[k]) {
                yob = a.out_ptr[x[k]];
                yod = a.out_ptr[x[k] + 1] - yob;
                const bool inb = (long long)(LLP_INF - cand[k]) < hi;
                if (!lq_put(sh, inb && yod > 0 && yod <= LQ_DEG, x[k], yob, yod)) {
                    lmin = min(lmin, dist_key(a, cand[k]));
                    changed = amax(&a.cstamp[x[k]], r) < r;
                }
            }
            if (changed) nadv++;
            append<COH>(changed && yod > 0, x[k], yob, yod, ctr, out, &a.ctrl->status);
        }
    }
    if (arcs) atomicAdd((unsigned long long*)&sh.lq_arcs, (unsigned long long)arcs);
}

// Delta buckets: an input entry whose vertex lies at distance >= hi is not
// expanded (or pushed from) this round but carried into CL[r].  The entry is
// carried by the lane holding it in the iteration where it starts; every edge
// lane learns whether its owner is carried.  Returns the owner's flag.
__device__ __forceinline__ bool carry_step(const GArgs& a, const EdgeCtx& c, int r, long long hi, const ListRef& cl,
                                           unsigned long long* ctr, GShared& sh) {
    if (hi <= 0) return false;
    bool carry = false;
    int dm = 0;
    if (c.mine_valid) {
        int v = guard(c.mine.x, a.n, a.ctrl->diag, 65);
        dm = LLP_INF - a.G[v];
        carry = (long long)dm >= hi;
    }
    const bool starts = c.mine_valid && c.mine.z >= c.base && c.mine.z < c.limit;
    const bool put = carry && starts;
    if (put) amax(&a.cstamp[guard(c.mine.x, a.n, a.ctrl->diag, 66)], r);
    append(put, c.mine.x, c.mine.y, c.mine.w, ctr, cl, &a.ctrl->status);
    if (cl.segmin) wave_min_to_lds(put, dm, &sh.cmin);
    const int k = __popcll(ballot(put));
    if (lane() == 0 && k && a.trace) atomicAdd(&sh.carried, k);
    return shfl(carry ? 1 : 0, c.j) != 0;
}

// Expansion: stamp out-neighbours for round r and append new candidates to WL.
__device__ __forceinline__ void expand_body(const GArgs& a, const EdgeCtx& c, int r, GShared& sh, bool skip) {
    bool fresh = false;
    int x = 0, rb = 0, d = 0;
    if (c.active && !skip) {
        x = guard(a.out_dst[guard(c.csr, a.m, a.ctrl->diag, 51, c.own.y, c.own.z)], a.n, a.ctrl->diag, 52);
        if (a.stamp[x] < r && amax(&a.stamp[x], r) < r) {
            rb = a.in_ptr[x];
            d = a.in_ptr[x + 1] - rb;
            fresh = d > 0;
        }
    }
    append(fresh, x, rb, d, &sh.ctr, a.wl, &a.ctrl->status);
}

__device__ __forceinline__ void wave_range(int total, int& wb, int& we) {
    const long long W = (long long)gridDim.x * GW;
    const long long w = (long long)blockIdx.x * GW + (threadIdx.x >> 6);
    wb = (int)((long long)total * w / W);
    we = (int)((long long)total * (w + 1) / W);
}

template <bool COH = false>
__device__ __forceinline__ void publish(const ListRef& out, unsigned long long ctr, int cmin) {
    st_u64<COH>(out.seg + blockIdx.x, ctr);
    if (out.segmin) st_i32<COH>(out.segmin + blockIdx.x, cmin);
}

// Delta width of a round code (0: no buckets).
__device__ __forceinline__ int delta_of(const GArgs& a, int code) {
    const int mode = code & 3, dc = (code >> 8) & 3;
    if (a.jobs || mode == MODE_DENSE) return 0;
    const int base = a.ctrl->dbase > 0 ? a.ctrl->dbase : 1;
    switch (dc) {
        case DCLS_BASE: return base;
        case DCLS_WIDE: return base <= (1 << 24) ? base * 64 : (1 << 30);
        case DCLS_EXPLICIT: return a.sp.delta;
        default: return 0;
    }
}

__device__ int dense_cap(const GArgs& a, int r, GShared& sh);

// PRE launch of a BFS dense round r evaluated with the bitmap (cap = INF -
// (dmin + 1), dmin the smallest distance in CL[r-1]).  Bit v of a.bm is set
// iff d(v) <= dmin: such a tail offers its head exactly the cap, which bounds
// every row this round, and a tail with a larger distance offers less.  The
// round evaluates only the marked tails; an entry of CL[r-1] above dmin is
// carried into CL[r] instead, so each of its arcs that this round leaves
// unsatisfied keeps its tail listed (invariant I), and an unlisted tail's
// arcs are satisfied already.  Marks do not change within the round: rows
// advance to dmin + 1 at most.
constexpr int BM_SCAN = 16;    // bitmap words per wave per pass
constexpr int BM_CARRY = 8;    // list entries per thread per pass
__device__ void bm_prepare(const GArgs& a, int r, int cap, const ListRef& in, const ListRef& out, GShared& sh) {
    const int l = lane();
    const long long words = ((long long)a.n + 63) >> 6;
    const long long W = (long long)gridDim.x * GW;
    // 16 words per wave in flight: the scan is one or two passes
    for (long long c = (long long)blockIdx.x * GW + (threadIdx.x >> 6); c < words; c += BM_SCAN * W) {
        int g[BM_SCAN];
#pragma unroll
        for (int j = 0; j < BM_SCAN; ++j) {
            const long long v = (c + j * W) * 64 + l;
            g[j] = v < a.n ? a.G[v] : 0;
        }
#pragma unroll
        for (int j = 0; j < BM_SCAN; ++j) {
            const unsigned long long b = ballot(g[j] > cap);
            if (l == 0 && c + j * W < words) a.bm[c + j * W] = b;
        }
    }
    const int cnt = min(sh.cnt[blockIdx.x], in.cap);
    const int4* ent = in.ent + (long long)blockIdx.x * in.cap;
    int dmn = LLP_INF;
    for (int base = 0; base < cnt; base += BM_CARRY * GB) {
        int4 e[BM_CARRY];
        int g[BM_CARRY];
#pragma unroll
        for (int j = 0; j < BM_CARRY; ++j) {
            const int i = base + j * GB + (int)threadIdx.x;
            e[j] = i < cnt ? ent[i] : make_int4(-1, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < BM_CARRY; ++j) g[j] = e[j].x >= 0 ? a.G[guard(e[j].x, a.n, a.ctrl->diag, 68)] : LLP_INF;
#pragma unroll
        for (int j = 0; j < BM_CARRY; ++j) {
            const bool put = e[j].x >= 0 && g[j] <= cap;   // d > dmin
            if (put) {
                amax(&a.cstamp[guard(e[j].x, a.n, a.ctrl->diag, 68)], r);
                dmn = min(dmn, LLP_INF - g[j]);
            }
            append(put, e[j].x, e[j].y, e[j].w, &sh.ctr, out, &a.ctrl->status);
            const int nput = __popcll(ballot(put));
            if (l == 0 && nput && a.trace) atomicAdd(&sh.carried, nput);
        }
    }
    if (out.segmin) wave_min_to_lds(true, dmn, &sh.cmin);
    __syncthreads();
    if (threadIdx.x == 0) {
        publish(out, sh.ctr, sh.cmin);   // MAIN appends after the carried entries
        if (sh.carried) atomicAdd(&a.ctrl->carried[r & 1], sh.carried);
    }
}

// --------------------------------------------------------------- PRE
// Round r, first phase: consume CL[r-1], decide the round's code, then
// expand into WL (pull) or push (CL[r]); returns the code of a dense round,
// whose evaluation follows in the same launch, else -1.  k: step launch.
// BM: a bounded BFS dense round prepares the bitmap here and is evaluated by
// the next launch.
template <bool LQ, bool BM>
__device__ __forceinline__ int pre_phase(const GArgs& a, int r, int k, GShared& sh, const SegRegs& sin) {
    const ListRef in = cl_of(a, r - 1);
    const ListRef out = cl_of(a, r);
    // the learned schedule's inputs besides the list totals (its weights and
    // the previous round's record) are read before the totals are scanned
    MlpLane wl{};
    SchedHist hprev{};
    if (a.sp.sched == LLP_SCHED_LEARNED && a.sp.mlp && threadIdx.x < 64) {
        wl = mlp_load(a.sp.mlp);
        hprev = a.ctrl->hist[(r + 1) & 1];
    }
    seg_scan(sin, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);   // totals of CL[r-1]
    const int force_dense = (r == 1 && a.warm_dense);
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.trace && r >= 2 && r - 2 < a.trace_cap) {
        // entries the previous round's delta filter carried
        a.trace[r - 2].pending = a.ctrl->carried[(r - 1) & 1];
        a.ctrl->carried[(r - 1) & 1] = 0;
    }
    if (sh.tot_count == 0 && !force_dense) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.ctrl->done = 1;
            a.ctrl->last_round = r - 1;
            a.ctrl->end_k = k;
            st_relaxed(&a.ctrl->stop[(k + 1) & 1], 1);
        }
        // the sweep has ended: every workgroup sees it, and no other launch
        // touches G any more, so the output is decoded here (unless a
        // candidate overflowed: the overflow check reads the encoded states)
        if (a.fuse_end && !ld_relaxed(&a.ctrl->ovf)) {
            for (long long v = blockIdx.x * (long long)GB + threadIdx.x; v < a.n; v += (long long)gridDim.x * GB) {
                const int g = a.G[v];
                a.G[v] = g > 0 ? LLP_INF - g : LLP_INF;
            }
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->decoded = 1;
        }
        return -1;
    }
    if ((long long)r > a.max_rounds) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.ctrl->over = 1;
            a.ctrl->done = 1;
            a.ctrl->last_round = r - 1;
            st_relaxed(&a.ctrl->stop[(k + 1) & 1], 1);
        }
        return -1;
    }
    // schedule decision (identical in every workgroup)
    if (threadIdx.x < 64) {
        int code = decide_mode(a.sp, hprev, r, sh.tot_count, sh.tot_edges, a.n, a.m,
                               force_dense, wl, reinterpret_cast<float*>(sh.own[0]));
        if (threadIdx.x == 0) sh.code = code;
    }
    if (threadIdx.x == 0) {
        sh.ctr = 0ull;
        sh.cctr = 0ull;
        sh.cmin = LLP_INF;
        sh.carried = 0;
        sh.lq_top = 0;
        sh.lq_arcs = 0;
    }
    __syncthreads();
    const int code = sh.code;
    const int mode = code & 3;
    const int delta = delta_of(a, code);
    long long hi = 0;   // bucket ceiling (distance), 0 = no buckets
    if (delta > 0 && in.segmin) {
        const int dmin = load_segmin(in.segmin, a.nseg, &sh.tmp1);
        hi = ((long long)dmin / delta) * delta + delta;
    }
    // the same bound the evaluation computes from the same list (dense_cap)
    const int bcap = (BM && mode == MODE_DENSE && !(r == 1 && a.warm_dense)) ? dense_cap(a, r, sh) : LLP_INF;
    const bool bmr = bcap != LLP_INF;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        GCtrl* c = a.ctrl;
        c->mode = code;
        c->rounds = r;
        // the next step launch: MAIN of a pull round or of a bitmap dense
        // round, else PRE of the next round (a dense round is evaluated in
        // this launch)
        c->step_phase[(k + 1) & 1] = mode == MODE_PULL ? 1 : (bmr ? 2 : 0);
        c->step_round[(k + 1) & 1] = r;
        if (a.plog && k < a.plog_cap) a.plog[k] = 0;
        c->adv += sh.tot_count;
        if (bmr) c->bmr++;
        if (mode == MODE_PULL) c->xedges += sh.tot_edges;
        if (mode == MODE_PUSH) c->pedges += sh.tot_edges;
        hist_push(c->hist[r & 1], c->hist[(r + 1) & 1], r, mode, sh.tot_count, sh.tot_edges);
        if (a.trace && r - 1 < a.trace_cap) {
            llp_trace_rec t;
            t.round = r;
            t.mode = code;
            t.in_count = sh.tot_count;
            t.out_count = 0;
            t.in_edges = sh.tot_edges;
            t.out_edges = 0;
            t.bucket = hi > 0 ? (int)(hi - delta) : -1;
            t.pending = 0;
            t.bitmap = bmr ? 1 : 0;
            t.pad = 0;
            a.trace[r - 1] = t;
        }
    }
    if (mode == MODE_DENSE) {
        if (bmr) {
            bm_prepare(a, r, bcap, in, out, sh);
            return -1;
        }
        return code;   // evaluated by the caller in this launch
    }
    SegView sv{in.ent, in.cap, a.nseg, sh.cnt, sh.epre, sh.tot_edges, sh.tot_count};
    ListSrc src{sv, a.ctrl->diag};
    int wb, we;
    wave_range(sh.tot_edges, wb, we);
    int* own = sh.own[threadIdx.x >> 6];
    bool ovf = false;
    long long nadv = 0;
    if (mode == MODE_PULL) {
        for_edges(src, wb, we, own, [&](const EdgeCtx& c) {
            bool skip = carry_step(a, c, r, hi, out, &sh.cctr, sh);
            expand_body(a, c, r, sh, skip);
        });
        __syncthreads();
        if (threadIdx.x == 0) {
            publish(a.wl, sh.ctr, LLP_INF);
            publish(out, sh.cctr, sh.cmin);   // MAIN appends after the carried entries
        }
    } else {
        int lmin = LLP_INF;
        push_wave<false, LQ>(a, src, wb, we, r, hi, out, &sh.ctr, sh, sh.pw[threadIdx.x >> 6], ovf, nadv, lmin);
        if constexpr (LQ) {
            if (hi > 0 && !a.jobs) local_drain<false>(a, r, hi, out, &sh.ctr, sh, ovf, nadv, lmin);
        }
        if (out.segmin) wave_min_to_lds(true, lmin, &sh.cmin);
        __syncthreads();
        if (threadIdx.x == 0) {
            publish(out, sh.ctr, sh.cmin);
            if (sh.lq_arcs) atomicAdd((unsigned long long*)&a.ctrl->pedges, (unsigned long long)sh.lq_arcs);
        }
    }
    if (threadIdx.x == 0 && sh.carried) atomicAdd(&a.ctrl->carried[r & 1], sh.carried);
    if (__any(ovf) && lane() == 0) st_relaxed(&a.ctrl->ovf, 1);
    return -1;
}

// Bound for the dense round r of a BFS: with dmin the smallest distance in
// CL[r-1], every vertex whose distance is not final has true distance
// >= dmin + 1 (on a shortest path to it, the last vertex with a final
// distance has an out-arc still to propagate, so it is in CL[r-1]), and
// states never pass the fixpoint.  So a candidate INF - (dmin + 1) is the
// largest any row can still take (its evaluation may stop there), and a row
// already at or above it is final.  LLP_INF (no bound) elsewhere: weighted
// graphs (the smallest weight is unknown), jobs, verification.
__device__ int dense_cap(const GArgs& a, int r, GShared& sh) {
    if (!a.unit_w || a.jobs) return LLP_INF;
    const ListRef in = cl_of(a, r - 1);
    if (!in.segmin) return LLP_INF;
    const int dmin = load_segmin(in.segmin, a.nseg, &sh.tmp1);
    return dmin < LLP_INF - 1 ? LLP_INF - (dmin + 1) : LLP_INF;
}

// Smallest distance dlo in CL[r-1] for the arc bound of a weighted dense
// round.  By invariant I (an arc (u, v) either satisfies d(v) <= d(u) + w
// or has u in CL[r-1]), an arc can improve v this round only if its tail is
// in CL[r-1], so d(u) >= dlo, and only if dlo + w < d(v): arcs failing that
// are not gathered.  An arc skipped while its tail improves during the
// round is seen again in the next round, the tail being listed in CL[r].
// -1 (no bound): unit weights (dense_cap covers them), jobs, verification.
__device__ int dense_dmin(const GArgs& a, int r, GShared& sh) {
    if (a.unit_w || a.jobs) return -1;
    const ListRef in = cl_of(a, r - 1);
    if (!in.segmin) return -1;
    const int dmin = load_segmin(in.segmin, a.nseg, &sh.tmp1);
    return dmin < LLP_INF - 1 ? dmin : -1;
}

// --------------------------------------------------------------- MAIN
// Round r, second phase (pull and dense rounds): evaluate WL (or every
// vertex) and produce CL[r].  verify != 0: a dense round on the final state
// that must change nothing.
// bmr: a BFS dense round whose PRE launch built the bitmap and carried the
// entries above dmin into CL[r] (this launch appends after them); BM: the
// kernel evaluates every dense round so (see bm_prepare).
template <bool BM>
__device__ __forceinline__ void main_phase(const GArgs& a, int r, int verify, int k, GShared& sh, int round_code, bool bmr) {
    const int code = verify ? MODE_DENSE : round_code;
    const int mode = code & 3;
    if (!verify && blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctrl->step_phase[(k + 1) & 1] = 0;
        a.ctrl->step_round[(k + 1) & 1] = r;
        if (a.plog && k < a.plog_cap) a.plog[k] = 1;
    }
    if (mode == MODE_PUSH) return;
    const ListRef out = verify ? a.wl : cl_of(a, r);   // verify writes into WL's storage
    if (threadIdx.x == 0) {
        // pull rounds (and bitmap rounds) continue the segment PRE started with carried entries
        const bool cont = (mode == MODE_PULL || bmr) && !verify;
        sh.ctr = cont ? out.seg[blockIdx.x] : 0ull;
        sh.cmin = (cont && out.segmin) ? out.segmin[blockIdx.x] : LLP_INF;
        sh.cnt_rd = 0ull;
        sh.cnt_gath = 0ull;
    }
    int* own = sh.own[threadIdx.x >> 6];
    bool ovf = false;
    long long nadv = 0;
    int wb, we;
    if (mode == MODE_DENSE) {
        __syncthreads();
        const bool bounded = !verify && !(r == 1 && a.warm_dense);
        const int cap = bounded ? dense_cap(a, r, sh) : LLP_INF;
        const int dlo = bounded ? dense_dmin(a, r, sh) : -1;
        if (blockIdx.x == 0 && threadIdx.x == 0 && !verify) {
            a.ctrl->cand += a.n;
            if (cap == LLP_INF && dlo < 0) {   // with a bound, the waves count what they read
                a.ctrl->edges += a.m;
                a.ctrl->gath += a.m;
            }
        }
        int rr = verify ? r + 1 : r;
        wave_range(a.m, wb, we);
        int lmin = LLP_INF;
        int nrd = 0, nins = 0;
        if (BM && !bmr && !verify) {
            // the bitmap kernel runs only sweeps whose dense rounds are all
            // bounded (BFS without a warm start): an unbounded one is a fault
            if (blockIdx.x == 0 && threadIdx.x == 0) set_status(&a.ctrl->status, LLP_E_HIP);
        } else {
            dense_wave<BM>(a, rr, wb, we, out, sh, sh.dcb[threadIdx.x >> 6], ovf, nadv, lmin, cap, dlo, nrd, nins);
        }
        if ((cap != LLP_INF || dlo >= 0) && !verify) {
            // arcs read and states gathered: summed per workgroup in LDS, one
            // atomic each per workgroup
            const long long rd = wave_sum64(nrd), tot = wave_sum64(nins);
            if (lane() == 0) {
                atomicAdd(&sh.cnt_rd, (unsigned long long)rd);
                atomicAdd(&sh.cnt_gath, (unsigned long long)tot);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                if (sh.cnt_rd) atomicAdd((unsigned long long*)&a.ctrl->edges, sh.cnt_rd);
                if (sh.cnt_gath) atomicAdd((unsigned long long*)&a.ctrl->gath, sh.cnt_gath);
            }
        }
        if (out.segmin) wave_min_to_lds(true, lmin, &sh.cmin);
    } else {
        load_segments(a.wl.seg, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.ctrl->cand += sh.tot_count;
            a.ctrl->edges += sh.tot_edges;
            a.ctrl->gath += sh.tot_edges;
            a.ctrl->hist[r & 1].wl_count = sh.tot_count;
            a.ctrl->hist[r & 1].wl_edges = sh.tot_edges;
            if (a.trace && r - 1 < a.trace_cap) {
                a.trace[r - 1].out_count = sh.tot_count;
                a.trace[r - 1].out_edges = sh.tot_edges;
            }
        }
        SegView sv{a.wl.ent, a.wl.cap, a.nseg, sh.cnt, sh.epre, sh.tot_edges, sh.tot_count};
        ListSrc src{sv, a.ctrl->diag};
        wave_range(sh.tot_edges, wb, we);
        for_edges(src, wb, we, own, [&](const EdgeCtx& c) { eval_body(a, c, r, out, sh, ovf, nadv); });
    }
    __syncthreads();
    if (threadIdx.x == 0) publish(out, sh.ctr, sh.cmin);
    if (__any(ovf) && lane() == 0) st_relaxed(&a.ctrl->ovf, 1);
    if (verify) {
        long long tot = wave_sum64(nadv);
        if (lane() == 0 && tot) st_relaxed(&a.ctrl->verify_changed, 1);
    }
}

// One step of the sweep: launch k runs the phase the previous launch left in
// slot k & 1 (PRE of the next round, or MAIN of the current one).  A dense
// round is decided and evaluated in one launch (every workgroup takes the
// same decision from the same list totals), so push and dense rounds cost
// one launch, a pull round two.  The slots alternate, so no workgroup of
// launch k reads the slot launch k writes.  The same holds for the stop
// word: the launch that finds the end (and decodes G, every workgroup its
// share) sets stop[(k + 1) & 1] for the launches after it, each of which
// passes it on; a workgroup of the finishing launch that starts late must
// not see it, or its share of G would be left encoded.  LQ: the local
// queues of bucketed push rounds are compiled in (launched when a solve can
// have bucketed rounds; without them a bucketed push round continues chains
// instead, and the kernel is smaller, which the dense rounds measurably
// prefer).
template <bool LQ, bool BM>
__global__ void __launch_bounds__(GB, 4) k_graph_step(GArgs a, int k) {
    __shared__ GShared sh;
    // one round trip for the launch's control words and the totals of both
    // changed lists (the round's parity picks one)
    SegRegs s0, s1;
    seg_fetch(a.cl0.seg, a.nseg, s0);
    seg_fetch(a.cl1.seg, a.nseg, s1);
    const int ph = a.ctrl->step_phase[k & 1];
    const int rr = a.ctrl->step_round[k & 1];
    if (ld_relaxed(&a.ctrl->stop[k & 1]) || ld_relaxed(&a.ctrl->status)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_relaxed(&a.ctrl->stop[(k + 1) & 1], 1);
        return;
    }
    int r = rr, code;
    if (ph == 0) {
        r = rr + 1;
        code = pre_phase<LQ, BM>(a, r, k, sh, (rr & 1) ? s1 : s0);   // CL[r-1] = CL[rr]
        if (code < 0) return;
    } else {
        code = a.ctrl->mode;
    }
    main_phase<BM>(a, r, 0, k, sh, code, ph == 2);
}

// --------------------------------------------------------------- tail
// Multi-round mode for narrow push rounds (the tail of a sweep, and every
// round of a bucketed sweep on a mesh, where a round pushes a few tens of
// thousands of arcs and a launch per round costs more than the round).  A
// cooperative launch of the step kernel's shape in which only the
// workgroups with blockIdx % TAIL_XCDS == 0 work: workgroups are dispatched
// round-robin over the XCDs, so these share one XCD's L2.  They run
// consecutive push rounds separated by a barrier on a counter.  Every list
// word they exchange within the launch (entries, segment totals and minima)
// is written and read by agent-scope atomics; states advance by atomicMax
// and are read by atomic loads where a stale value would be wrong (the value
// pushed), plain loads only as a precheck.  The barrier is correct wherever
// the workgroups run; only its speed depends on the placement.  The launch
// hands back to the step launches at the first round that is not a push
// round of at most TAIL_EDGES arcs (or that the learned network would
// decide), after TAIL_ROUNDS rounds, or at the end of the sweep, which it
// decodes; it reads and writes the step slot k & 1 of the step launch k
// that follows it.  Every wait is bounded: a barrier that does not complete
// within TAIL_SPIN polls sets LLP_E_HIP and ends the launch.
constexpr int TAIL_XCDS = 8;
constexpr int TAIL_EDGES = 1 << 17;
constexpr int TAIL_ROUNDS = 4096;
constexpr int TAIL_SPIN = 1 << 22;

__device__ bool tail_barrier(unsigned* bar, unsigned target, int* status, int* ok) {
    // every memory operation of the round, atomics without a used result and
    // atomic stores included, has completed before the count moves
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        *ok = 1;
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int spins = 0; __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target;) {
            if (++spins > TAIL_SPIN || ((spins & 1023) == 0 && ld_relaxed(status))) {
                set_status(status, LLP_E_HIP);
                *ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    return *ok != 0;
}

__global__ void __launch_bounds__(GB, 4) k_graph_tail(GArgs a, int k) {
    __shared__ GShared sh;
    if (blockIdx.x % TAIL_XCDS) return;
    GCtrl* c = a.ctrl;
    const int P = gridDim.x / TAIL_XCDS, me = blockIdx.x / TAIL_XCDS;
    const bool lead = me == 0 && threadIdx.x == 0;
    // no stop check here: the host launches the tail only after reading back a
    // sweep that has not ended, and a participant that starts after the lead
    // has found the end (and set the stop word for the next step launch) must
    // still decode its share
    if (ld_relaxed(&c->status) || ld_relaxed(&c->step_phase[k & 1]) != 0) return;
    int r = ld_relaxed(&c->step_round[k & 1]) + 1;
    const int wave = threadIdx.x >> 6;
    const long long W = (long long)P * GW, w = (long long)me * GW + wave;
    for (int t = 0;; ++t, ++r) {
        const ListRef in = cl_of(a, r - 1);
        const ListRef out = cl_of(a, r);
        load_segments<true>(in.seg, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);
        if (sh.tot_count == 0) {
            // the end of the sweep: decode G as the step launch that finds it does
            if (lead) {
                c->done = 1;
                c->last_round = r - 1;
                st_relaxed(&c->stop[k & 1], 1);
            }
            if (a.fuse_end && !ld_relaxed(&c->ovf)) {
                for (long long v = (long long)me * GB + threadIdx.x; v < a.n; v += (long long)P * GB) {
                    const int g = ld_relaxed(&a.G[v]);
                    a.G[v] = g > 0 ? LLP_INF - g : LLP_INF;
                }
                if (lead) c->decoded = 1;
            }
            return;
        }
        if ((long long)r > a.max_rounds) {
            if (lead) {
                c->over = 1;
                c->done = 1;
                c->last_round = r - 1;
                st_relaxed(&c->stop[k & 1], 1);
            }
            return;
        }
        const bool netround = a.sp.sched == LLP_SCHED_LEARNED &&
                              (long long)sh.tot_edges * LEARNED_MIN_FRAC >= (long long)a.m;
        if (threadIdx.x < 64) {
            // history records are not needed: the learned network's rounds hand back
            SchedHist none{};
            MlpLane wl{};
            const int code = netround ? round_code(MODE_PULL, DCLS_NONE)
                                      : decide_mode(a.sp, none, r, sh.tot_count, sh.tot_edges, a.n, a.m, 0, wl,
                                                    reinterpret_cast<float*>(sh.own[0]));
            if (threadIdx.x == 0) {
                sh.code = code;
                sh.ctr = 0ull;
                sh.cmin = LLP_INF;
                sh.carried = 0;
                sh.lq_top = 0;
                sh.lq_arcs = 0;
            }
        }
        __syncthreads();
        const int code = sh.code;
        // a round's appends (at most one per arc) must fit the participants' segments
        const bool fits = 2ll * sh.tot_edges <= (long long)P * out.cap;
        if ((code & 3) != MODE_PUSH || sh.tot_edges > TAIL_EDGES || !fits || t >= TAIL_ROUNDS) {
            // hand back: the next step launch runs PRE of round r
            if (lead) {
                c->step_phase[k & 1] = 0;
                c->step_round[k & 1] = r - 1;
            }
            return;
        }
        // the other workgroups' segments of the output list hold an older
        // round's totals: cleared in the first two rounds (one per list)
        if (t < 2) {
            for (int sg = me * GB + threadIdx.x; sg < a.nseg; sg += P * GB) {
                if (sg % TAIL_XCDS == 0) continue;
                st_u64<true>(out.seg + sg, 0ull);
                st_i32<true>(out.segmin + sg, LLP_INF);
            }
        }
        const int delta = delta_of(a, code);
        long long hi = 0;
        if (delta > 0) {
            const int dmin = load_segmin<true>(in.segmin, a.nseg, &sh.tmp1);
            hi = ((long long)dmin / delta) * delta + delta;
        }
        if (lead) {
            c->mode = code;
            c->rounds = r;
            c->tail_rounds++;
            c->adv += sh.tot_count;
            c->pedges += sh.tot_edges;
            hist_push(c->hist[r & 1], c->hist[(r + 1) & 1], r, MODE_PUSH, sh.tot_count, sh.tot_edges);
            if (a.trace && r - 1 < a.trace_cap) {
                if (r >= 2 && r - 2 < a.trace_cap) {
                    a.trace[r - 2].pending = c->carried[(r - 1) & 1];
                    c->carried[(r - 1) & 1] = 0;
                }
                llp_trace_rec tr;
                tr.round = r;
                tr.mode = code;
                tr.in_count = sh.tot_count;
                tr.out_count = 0;
                tr.in_edges = sh.tot_edges;
                tr.out_edges = 0;
                tr.bucket = hi > 0 ? (int)(hi - delta) : -1;
                tr.pending = 0;
                tr.bitmap = 0;
                tr.pad = 0;
                a.trace[r - 1] = tr;
            }
        }
        SegView sv{in.ent, in.cap, a.nseg, sh.cnt, sh.epre, sh.tot_edges, sh.tot_count};
        ListSrcT<true> src{sv, c->diag};
        const int wb = (int)((long long)sh.tot_edges * w / W), we = (int)((long long)sh.tot_edges * (w + 1) / W);
        bool ovf = false;
        long long nadv = 0;
        int lmin = LLP_INF;
        push_wave<true, true>(a, src, wb, we, r, hi, out, &sh.ctr, sh, sh.pw[wave], ovf, nadv, lmin);
        if (hi > 0) local_drain<true>(a, r, hi, out, &sh.ctr, sh, ovf, nadv, lmin);
        wave_min_to_lds(true, lmin, &sh.cmin);
        __syncthreads();
        if (threadIdx.x == 0) {
            publish<true>(out, sh.ctr, sh.cmin);
            if (sh.lq_arcs) atomicAdd((unsigned long long*)&c->pedges, (unsigned long long)sh.lq_arcs);
        }
        if (threadIdx.x == 0 && sh.carried) atomicAdd(&c->carried[r & 1], sh.carried);
        if (__any(ovf) && lane() == 0) st_relaxed(&c->ovf, 1);
        if (!tail_barrier(&c->tail_bar, (unsigned)(t + 1) * (unsigned)P, &c->status, &sh.tmp1)) return;
    }
}

__global__ void k_graph_tail_reset(GCtrl* c) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c->tail_bar = 0u;
}

__global__ void __launch_bounds__(GB) k_graph_verify(GArgs a, int r) {
    __shared__ GShared sh;
    main_phase<false>(a, r, 1, 0, sh, MODE_DENSE, false);
}

// --------------------------------------------------------------- finish
// Overflow: a vertex still at the bottom with a reached in-neighbour has a
// true distance >= INF.  Only run when a candidate overflowed.
// Jobs: every completion time S[j] + dur[j] must fit int32 (always checked).
// after_done: enqueued behind a batch of step launches; does nothing unless
// the sweep has ended without error.
__global__ void k_graph_ovf(GArgs a, int after_done) {
    if (after_done && (!ld_relaxed(&a.ctrl->done) || ld_relaxed(&a.ctrl->status))) return;
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    if (a.jobs) {
        bool bad = false;
        for (long long v = tid; v < a.n; v += nt)
            if ((long long)a.G[v] + a.vdur[v] > LLP_INF) bad = true;
        if (bad) set_status(&a.ctrl->status, LLP_E_OVERFLOW);
        return;
    }
    if (!ld_relaxed(&a.ctrl->ovf)) return;
    for (long long v = tid; v < a.n; v += nt) {
        if (a.G[v] != 0) continue;
        bool bad = false;
        for (int e = a.in_ptr[v]; e < a.in_ptr[v + 1]; ++e)
            if (a.G[clampi(a.in_src[clampi(e, a.m, bad)], a.n, bad)] > 0) {
                set_status(&a.ctrl->status, LLP_E_OVERFLOW);
                break;
            }
    }
}

// In place: G -> distance (INF for unreached), after verification or an
// overflow check (otherwise the step launch that finds the end decodes).
__global__ void k_graph_decode(int* G, int n) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < n; v += nt) {
        int g = G[v];
        G[v] = g > 0 ? LLP_INF - g : LLP_INF;
    }
}

// --------------------------------------------------------------- host
struct GraphLayout {
    int nseg;
    int cap;
};

// per_cu: workgroups (= list segments) per CU, opts->chunk for graph solves;
// the default 2 keeps every workgroup of a phase kernel resident at once.
static int graph_wgs_per_cu(int chunk) { return chunk > 0 ? (chunk > 8 ? 8 : chunk) : 2; }
// workgroups per CU the autotuner tries (llp_autotune_graph); a solve that
// leaves the choice to the library (chunk 0) takes the record of its size
// class, so workspaces sized for chunk 0 hold every candidate
constexpr int GRAPH_TUNE_MAX = 4;

static GraphLayout graph_layout(int64_t m, int per_cu) {
    const DeviceInfo& d = device_info();
    GraphLayout L;
    L.nseg = d.cus * per_cu;
    if (L.nseg > MAX_SEG) L.nseg = MAX_SEG;
    long long W = (long long)L.nseg * GW;
    long long per_wave = (m + W - 1) / W;
    L.cap = (int)(GW * per_wave + GW * 2 + 64);
    return L;
}

static size_t graph_ws(int64_t n, int64_t m, int per_cu, GArgs* a, char* base, size_t cap) {
    GraphLayout L = graph_layout(m, per_cu);
    Carver cv{base, cap, 0, base == nullptr};
    int* stamp = cv.take<int>(n);
    int* cstamp = cv.take<int>(n);
    unsigned long long* bm = cv.take<unsigned long long>((n + 63) / 64);
    GCtrl* ctrl = cv.take<GCtrl>(1);
    const long long plog_cap = 8 * n + 512;   // covers the default round limit's launches
    signed char* plog = cv.take<signed char>(plog_cap);
    ListRef lists[3];
    for (int i = 0; i < 3; ++i) {
        // CL lists hold the entries a delta round carries plus the round's own
        // appends in one segment: twice the capacity
        const int cap = i == 0 ? L.cap : 2 * L.cap;
        lists[i].seg = cv.take<unsigned long long>(L.nseg);
        lists[i].segmin = i == 0 ? nullptr : cv.take<int>(L.nseg);
        lists[i].ent = cv.take<int4>((size_t)L.nseg * cap);
        lists[i].cap = cap;
    }
    if (a) {
        a->stamp = stamp;
        a->cstamp = cstamp;
        a->bm = bm;
        a->ctrl = ctrl;
        a->wl = lists[0];
        a->cl0 = lists[1];
        a->cl1 = lists[2];
        a->nseg = L.nseg;
        a->plog = plog;
        a->plog_cap = plog_cap;
    }
    return cv.used;
}

size_t graph_workspace_bytes(int64_t n, int64_t m, int chunk) {
    if (chunk > 0) return graph_ws(n, m, graph_wgs_per_cu(chunk), nullptr, nullptr, 0);
    size_t b = 0;
    for (int c = 1; c <= GRAPH_TUNE_MAX; ++c) b = std::max(b, graph_ws(n, m, c, nullptr, nullptr, 0));
    return b;
}

__global__ void k_fill_i8(signed char* p, long long n, signed char v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// LLP_TIMING events, created once per thread and device and reused by every
// solve (creating events per launch would cost more than short rounds).
static hipEvent_t timing_event(size_t i) {
    static thread_local std::map<int, std::vector<hipEvent_t>> pool;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<hipEvent_t>& v = pool[dev];
    while (v.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        v.push_back(e);
    }
    return v[i];
}

// Whether the device runs cooperative launches (the tail kernel needs all its
// workgroups resident), asked once per device.
static bool coop_supported() {
    static std::map<int, bool> known;
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(dev);
    if (it != known.end()) return it->second;
    int v = 0;
    const bool ok = hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && v != 0;
    known[dev] = ok;
    return ok;
}

// lq: the kernel with local queues; bm: BFS dense rounds with the bitmap
static void launch_step(const GArgs& a, int k, bool lq, bool bm, hipStream_t st) {
    if (lq) hipLaunchKernelGGL((k_graph_step<true, false>), dim3(a.nseg), dim3(GB), 0, st, a, k);
    else if (bm) hipLaunchKernelGGL((k_graph_step<false, true>), dim3(a.nseg), dim3(GB), 0, st, a, k);
    else hipLaunchKernelGGL((k_graph_step<false, false>), dim3(a.nseg), dim3(GB), 0, st, a, k);
}

static int launch_grid_1d(int64_t work) {
    int64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    int cap = device_info().cus * 8;
    return (int)(g < cap ? g : cap);
}

// The step launches the last sweep of the same graph arrays, kind and
// schedule needed (sweeps that ended in step launches only).  The next such
// sweep sizes its first batch from it, never above the default, so a
// repeated solve enqueues few launches past its end; a sweep that needs more
// pays one more readback.  Outputs do not depend on it.
using SweepKey = std::tuple<const void*, const void*, int, long long, int, unsigned, unsigned, int>;
static std::mutex g_hmu;
static std::map<SweepKey, int> g_hist;
// The delta base width sampled from a weight array (by its address and arc
// count): later solves of the same weights skip the sample, a chain of
// random loads on as many pages that otherwise sets the init launch's length.
// Only bucket widths depend on it, never a fixpoint.
static std::map<std::pair<const void*, long long>, int> g_dbase;
constexpr int FIRST_BATCH = 16;

// jobs != nullptr: the pull form of job scheduling (in-CSR = predecessor
// lists, out-CSR = successor lists, per-job durations), otherwise SSSP / BFS.
static int solve_graph_core(const llp_graph* g, int32_t source, int32_t* out, const llp_opts* opts, bool bfs,
                            const int* jobs_dur) {
    if (!g) return fail(LLP_E_ARG, "graph is NULL");
    if (!out) return fail(LLP_E_ARG, "output is NULL");
    if (g->n <= 0) return fail(LLP_E_ARG, "n must be positive (got %d)", g->n);
    if (g->m < 0 || g->m > (int64_t)0x7fffffff - (1 << 20)) return fail(LLP_E_ARG, "m out of range");
    if (source < 0 || source >= g->n) return fail(LLP_E_ARG, "source %d out of range [0, %d)", source, g->n);
    if (!g->in_ptr || (g->m > 0 && !g->in_src)) return fail(LLP_E_ARG, "in-CSR arrays are required");
    if (!bfs && !jobs_dur && g->m > 0 && !g->in_w) return fail(LLP_E_ARG, "SSSP needs in_w (use llp_solve_bfs for unit weights)");
    llp_opts o = opts_or_default(opts);
    hipStream_t st = (hipStream_t)o.stream;
    const bool need_out = true;
    if (need_out && (!g->out_ptr || (g->m > 0 && !g->out_dst)))
        return fail(LLP_E_ARG, "out-CSR (out_ptr, out_dst) is required for successor expansion");
    if (o.sched == LLP_SCHED_FIXED && (o.flags & LLP_PUSH) && !bfs && !jobs_dur && !g->out_w)
        return fail(LLP_E_ARG, "push rounds need out_w");
    if (o.sched > LLP_SCHED_SCRIPT) return fail(LLP_E_ARG, "unknown schedule %u", o.sched);

    GArgs a;
    memset(&a, 0, sizeof(a));
    a.n = g->n;
    a.m = (int)g->m;
    a.in_ptr = g->in_ptr;
    a.in_src = g->in_src;
    a.in_w = bfs ? nullptr : g->in_w;
    a.out_ptr = g->out_ptr;
    a.out_dst = g->out_dst;
    a.out_w = bfs ? nullptr : g->out_w;
    a.G = out;
    a.source = source;
    a.unit_w = bfs ? 1 : 0;
    a.jobs = jobs_dur ? 1 : 0;
    a.vdur = jobs_dur;
    a.trace = (o.flags & LLP_TRACE) ? o.trace_dev : nullptr;
    a.trace_cap = o.trace_cap;
    a.warm_dense = (o.warm_start || jobs_dur) ? 1 : 0;   // jobs: every index is a round-1 candidate
    a.fuse_end = (!(o.flags & LLP_VERIFY) && !jobs_dur) ? 1 : 0;
    const bool can_push = bfs || jobs_dur || g->out_w != nullptr;
    int s = sched_params(o, can_push, &a.sp);
    if (s) return s;
    hybrid_params(jobs_dur ? LLP_KIND_JOBS : (bfs ? LLP_KIND_BFS : LLP_KIND_SSSP), g->n, g->m, can_push, &a.sp);

    int per_cu = graph_wgs_per_cu(o.chunk);
    if (o.chunk <= 0 && !jobs_dur) {
        int tb = 0, tc = 0;
        if (tune_lookup(bfs ? LLP_KIND_BFS : LLP_KIND_SSSP, g->m, &tb, &tc)) per_cu = std::min(std::max(tc, 1), GRAPH_TUNE_MAX);
    }
    size_t need = graph_ws(g->n, g->m, per_cu, nullptr, nullptr, 0);
    void* ws = nullptr;
    s = get_workspace(o, need, &ws);
    if (s) return s;
    graph_ws(g->n, g->m, per_cu, &a, (char*)ws, need);

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = (o.flags & LLP_TIMING) && o.stats;
    if (timing) {
        ev0 = timing_event(0);
        ev1 = timing_event(1);
        if (!ev0 || !ev1) return fail(LLP_E_HIP, "hipEventCreate failed");
        LLP_HIP(hipEventRecord(ev0, st));
    }
    const std::pair<const void*, long long> wkey((const void*)a.in_w, (long long)g->m);
    if (!a.unit_w && !a.jobs && a.in_w) {
        std::lock_guard<std::mutex> lk(g_hmu);
        auto it = g_dbase.find(wkey);
        if (it != g_dbase.end()) a.dbase_known = it->second;
    }
    const int g1 = launch_grid_1d(g->n > g->m ? g->n : g->m);
    hipLaunchKernelGGL(k_graph_init, dim3(launch_grid_1d(g->n)), dim3(256), 0, st, a, o.warm_start);
    if (o.flags & LLP_VALIDATE) hipLaunchKernelGGL(k_graph_validate, dim3(g1), dim3(256), 0, st, a);
    LLP_HIP(hipGetLastError());

    // watchdog: a DAG of jobs converges within n rounds (the limit is also the
    // cycle test); delta buckets can add rounds per bucket, hence the wider
    // graph limit
    const int64_t max_rounds =
        o.max_rounds > 0 ? o.max_rounds : (jobs_dur ? (int64_t)g->n + 2 : 4 * (int64_t)g->n + 64);
    a.max_rounds = max_rounds;
    GCtrl h;
    memset(&h, 0, sizeof(h));
    // step launches: at most two per round; the first batch (16, or what the
    // last sweep of this graph and schedule needed) covers a typical R-MAT
    // sweep, then the batch doubles up to 64
    const int64_t max_launches = 2 * max_rounds + 4;
    int64_t k = 0;
    const SweepKey hkey(g->in_ptr, g->out_ptr, g->n, (long long)g->m, jobs_dur ? 2 : (bfs ? 1 : 0), o.sched,
                        o.flags & (LLP_PUSH | LLP_DENSE), o.delta);
    int batch = FIRST_BATCH;
    {
        std::lock_guard<std::mutex> lk(g_hmu);
        auto it = g_hist.find(hkey);
        if (it != g_hist.end()) batch = std::max(2, std::min(FIRST_BATCH, it->second + 1));
    }
    int status = LLP_OK;
    bool finished = false;           // overflow check and decode done inside the loop
    std::vector<hipEvent_t> evs;     // LLP_TIMING: one pair around each step launch
    // the step kernel with local queues where bucketed push rounds can occur
    const bool lq_kernel = !jobs_dur && (a.sp.push_dclass == DCLS_WIDE || o.sched == LLP_SCHED_RANDOM ||
                                         o.sched == LLP_SCHED_SCRIPT || (o.sched == LLP_SCHED_FIXED && o.delta > 0));
    // BFS sweeps: bounded dense rounds look tails up in a bitmap
    const bool bm_kernel = bfs && !jobs_dur && !lq_kernel && !o.warm_start;
    // the multi-round tail: push rounds (hybrid, fixed push, learned), graphs
    // whose grid splits evenly over the XCDs, a device with cooperative launches
    bool tail_ok = !jobs_dur && a.nseg % TAIL_XCDS == 0 && a.sp.can_push &&
                   (o.sched == LLP_SCHED_HYBRID || o.sched == LLP_SCHED_LEARNED ||
                    (o.sched == LLP_SCHED_FIXED && (o.flags & LLP_PUSH))) && coop_supported();
    float tail_ms = 0.f;
    int64_t tail_launches = 0;
    if (timing && a.plog) {
        hipLaunchKernelGGL(k_fill_i8, dim3(launch_grid_1d(a.plog_cap)), dim3(256), 0, st, a.plog, a.plog_cap,
                           (signed char)-1);
    }
    for (;;) {
        for (int i = 0; i < batch && k < max_launches; ++i, ++k) {
            if (timing) {
                hipEvent_t e0 = timing_event(2 + evs.size());
                hipEvent_t e1 = timing_event(3 + evs.size());
                if (!e0 || !e1) return fail(LLP_E_HIP, "hipEventCreate failed");
                LLP_HIP(hipEventRecord(e0, st));
                launch_step(a, (int)k, lq_kernel, bm_kernel, st);
                LLP_HIP(hipEventRecord(e1, st));
                evs.push_back(e0);
                evs.push_back(e1);
            } else {
                launch_step(a, (int)k, lq_kernel, bm_kernel, st);
            }
        }
        // without verification, the step launch that finds the end decodes
        // the output itself (jobs: the overflow check follows the batch and
        // acts only once the sweep has ended), so one readback both sees the
        // end and finds the output final
        const bool early = !(o.flags & LLP_VERIFY);
        if (early) {
            if (jobs_dur) hipLaunchKernelGGL(k_graph_ovf, dim3(g1), dim3(256), 0, st, a, 1);
            if (timing) LLP_HIP(hipEventRecord(ev1, st));
        }
        LLP_HIP(hipGetLastError());
        s = readback(st, a.ctrl, &h, sizeof(h));
        if (s) return s;
        if (h.done && early && (jobs_dur || h.decoded)) finished = true;
        if (h.status) break;
        if (h.done) {
            if (h.over) status = LLP_E_NOT_CONVERGED;
            break;
        }
        if (o.abort_host && *o.abort_host) { status = LLP_E_ABORTED; break; }
        if (k >= max_launches) { status = LLP_E_NOT_CONVERGED; break; }
        if (batch < 64) batch *= 2;
        // the last round was a narrow push round: run the next rounds in the tail
        const SchedHist& last = h.hist[h.rounds & 1];
        if (tail_ok && (h.mode & 3) == MODE_PUSH && last.cl_edges <= TAIL_EDGES) {
            hipLaunchKernelGGL(k_graph_tail_reset, dim3(1), dim3(64), 0, st, a.ctrl);
            hipEvent_t t0 = timing ? timing_event(2 + evs.size()) : nullptr;
            hipEvent_t t1 = timing ? timing_event(3 + evs.size()) : nullptr;
            if (timing) LLP_HIP(hipEventRecord(t0, st));
            int kk = (int)k;
            void* args[] = {&a, &kk};
            if (hipLaunchCooperativeKernel(k_graph_tail, dim3(a.nseg), dim3(GB), args, 0, st) !=
                hipSuccess) {
                (void)hipGetLastError();
                tail_ok = false;   // the grid cannot be resident at once: step launches only
                continue;
            }
            if (timing) LLP_HIP(hipEventRecord(t1, st));
            s = readback(st, a.ctrl, &h, sizeof(h));
            if (s) return s;
            ++tail_launches;
            if (timing) {
                float ms = 0.f;
                LLP_HIP(hipEventElapsedTime(&ms, t0, t1));
                tail_ms += ms;
            }
            if (h.done && early && h.decoded) finished = true;
            if (h.status) break;
            if (h.done) {
                if (h.over) status = LLP_E_NOT_CONVERGED;
                break;
            }
        }
    }
    if (!finished) {
        if (status == LLP_OK && h.status == 0 && (o.flags & LLP_VERIFY)) {
            hipLaunchKernelGGL(k_graph_verify, dim3(a.nseg), dim3(GB), 0, st, a, (int)h.last_round + 1);
        }
        if (h.status == 0) hipLaunchKernelGGL(k_graph_ovf, dim3(g1), dim3(256), 0, st, a, 0);
        if (!jobs_dur)
            hipLaunchKernelGGL(k_graph_decode, dim3(launch_grid_1d(g->n)), dim3(256), 0, st, out, g->n);
        LLP_HIP(hipGetLastError());
        if (timing) LLP_HIP(hipEventRecord(ev1, st));
        s = readback(st, a.ctrl, &h, sizeof(h));
        if (s) return s;
    }
    if (h.done && !h.over && h.status == 0 && tail_launches == 0 && h.end_k >= 0) {
        std::lock_guard<std::mutex> lk(g_hmu);
        if (g_hist.size() >= 256) g_hist.clear();
        g_hist[hkey] = h.end_k + 1;
    }
    if (!a.unit_w && !a.jobs && a.in_w && a.dbase_known <= 0 && h.dbase > 0) {
        std::lock_guard<std::mutex> lk(g_hmu);
        if (g_dbase.size() >= 256) g_dbase.clear();
        g_dbase[wkey] = h.dbase;
    }
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = h.rounds;
        o.stats->candidates = h.cand;
        o.stats->edges_inspected = h.edges;
        o.stats->states_gathered = h.gath;
        o.stats->bitmap_rounds = h.bmr;
        o.stats->advances = h.adv;
        o.stats->expand_edges = h.xedges;
        o.stats->push_edges = h.pedges;
        if (timing) {
            const size_t nl = evs.size() / 2;
            std::vector<signed char> ph(nl, -1);
            if (a.plog && nl) {
                s = readback(st, a.plog, ph.data(), std::min<size_t>(nl, (size_t)a.plog_cap));
                if (s) return s;
            }
            float ms = 0.f, kms = 0.f, pms = 0.f;
            LLP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            for (size_t i = 0; i < nl; ++i) {
                float t = 0.f;
                LLP_HIP(hipEventElapsedTime(&t, evs[2 * i], evs[2 * i + 1]));
                if (ph[i] == 1) {
                    kms += t;
                    o.stats->eval_launches++;
                } else if (ph[i] == 0) {
                    pms += t;
                    o.stats->pre_launches++;
                }
            }
            o.stats->device_ms = ms;
            o.stats->kernel_ms = kms;
            o.stats->pre_ms = pms + tail_ms;   // a tail launch runs push rounds
            o.stats->pre_launches += tail_launches;
        }
    }
    if (h.diag[0]) {
        return fail(LLP_E_INPUT, "index guard %d fired: index %d bound %d context %d %d (round %lld)", h.diag[0],
                    h.diag[1], h.diag[2], h.diag[3], h.diag[4], h.rounds);
    }
    if (h.status) {
        if (h.status == LLP_E_INPUT) return fail(LLP_E_INPUT, "device validation rejected the graph");
        if (h.status == LLP_E_OVERFLOW)
            return fail(LLP_E_OVERFLOW, jobs_dur ? "a completion time does not fit int32"
                                                 : "a reachable distance does not fit int32");
        return fail(h.status, "device status %d", h.status);
    }
    if (h.verify_changed) return fail(LLP_E_HIP, "verification round advanced an index after convergence");
    if (status == LLP_E_NOT_CONVERGED && jobs_dur && o.max_rounds <= 0)
        return fail(LLP_E_CYCLE, "no fixpoint within n + 2 rounds: the job arcs contain a cycle");
    if (status == LLP_E_NOT_CONVERGED) return fail(status, "not converged after %lld rounds", (long long)max_rounds);
    if (status == LLP_E_ABORTED) return fail(status, "aborted by the host flag");
    return LLP_OK;
}

int solve_graph(const llp_graph* g, int32_t source, int32_t* out, const llp_opts* opts, bool bfs) {
    return solve_graph_core(g, source, out, opts, bfs, nullptr);
}

// Job scheduling, pull form: the generic sweep with alpha(S, j) = max over
// predecessors p of S[p] + dur[p], every job a round-1 candidate.  A DAG
// reaches its fixpoint within n rounds (each round is at least a Jacobi
// step), so the round limit doubles as the cycle test; a cycle of zero
// durations has a fixpoint and is not reported.
int solve_jobs_pull(int32_t n, const int32_t* pred_ptr, const int32_t* pred_idx, const int32_t* dur,
                    const int32_t* succ_ptr, const int32_t* succ_idx, int32_t* start, const llp_opts* opts,
                    int64_t E) {
    llp_graph g;
    memset(&g, 0, sizeof(g));
    g.n = n;
    g.m = E;
    g.in_ptr = pred_ptr;
    g.in_src = pred_idx;
    g.in_w = nullptr;
    g.out_ptr = succ_ptr;
    g.out_dst = succ_idx;
    g.out_w = nullptr;
    return solve_graph_core(&g, 0, start, opts, false, dur);
}

// Time the sweep at each workgroup count per CU (1 .. GRAPH_TUNE_MAX) on this
// graph with the caller's schedule: median of 3 solves after a warm-up, HIP
// events around each (every solve ends with its readback); record the fastest
// for (kind, size class of m).
int autotune_graph(const llp_graph* g, int32_t source, int32_t kind, int32_t* out, char* report,
                   size_t report_bytes, const llp_opts* opts) {
    if (kind != LLP_KIND_SSSP && kind != LLP_KIND_BFS) return fail(LLP_E_ARG, "kind must be LLP_KIND_SSSP or LLP_KIND_BFS");
    if (!g) return fail(LLP_E_ARG, "graph is NULL");
    llp_opts o = opts_or_default(opts);
    o.flags &= ~(LLP_ASYNC | LLP_TIMING | LLP_TRACE);
    o.stats = nullptr;
    hipStream_t st = (hipStream_t)o.stream;
    hipEvent_t e0, e1;
    LLP_HIP(hipEventCreate(&e0));
    LLP_HIP(hipEventCreate(&e1));
    std::string rep;
    float best_ms = 1e30f;
    int best_c = 0, s = LLP_OK;
    for (int c = 1; c <= GRAPH_TUNE_MAX && s == LLP_OK; ++c) {
        llp_opts oc = o;
        oc.chunk = c;
        std::vector<float> ts;
        for (int r = 0; r < 4 && s == LLP_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) s = fail(LLP_E_HIP, "hipEventRecord failed");
            if (s == LLP_OK) s = solve_graph(g, source, out, &oc, kind == LLP_KIND_BFS);
            if (s == LLP_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                s = fail(LLP_E_HIP, "timing events failed");
            float ms = 0.f;
            if (s == LLP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = fail(LLP_E_HIP, "hipEventElapsedTime failed");
            if (s == LLP_OK && r > 0) ts.push_back(ms);
        }
        if (s) break;
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        char line[64];
        snprintf(line, sizeof(line), "%d %.4f\n", c, med);
        rep += line;
        if (med < best_ms) {
            best_ms = med;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    tune_record(kind, g->m, 0, best_c);
    if (report && report_bytes) {
        const size_t k = rep.size() < report_bytes - 1 ? rep.size() : report_bytes - 1;
        memcpy(report, rep.data(), k);
        report[k] = 0;
    }
    return LLP_OK;
}

}  // namespace llp

extern "C" {

int llp_autotune_graph(const llp_graph* g, int32_t source, int32_t kind, int32_t* out, char* report,
                       size_t report_bytes, const llp_opts* opts) {
    return llp::autotune_graph(g, source, kind, out, report, report_bytes, opts);
}

int llp_solve_sssp(const llp_graph* g, int32_t source, int32_t* dist, const llp_opts* opts) {
    return llp::solve_graph(g, source, dist, opts, false);
}

int llp_solve_bfs(const llp_graph* g, int32_t source, int32_t* level, const llp_opts* opts) {
    return llp::solve_graph(g, source, level, opts, true);
}

}  // extern "C"
