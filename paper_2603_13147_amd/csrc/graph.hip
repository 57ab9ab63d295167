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
// `done` flag; later kernels return at once.  The host polls the flag every
// few rounds.
#include <string.h>

#include <algorithm>
#include <map>
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
    int carried[2];     // entries carried by the delta filter, by round parity (traced solves)
    int step_phase[2];  // step kernel k: phase[k & 1] 0 = PRE of round step_round + 1, 1 = MAIN of step_round
    int step_round[2];
    int diag[8];        // first guard event: site, index, bound, context
    long long rounds, cand, edges, adv, xedges, pedges;
    SchedHist hist[2];  // scheduler history, double-buffered by round parity
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
    GCtrl* ctrl;
    llp_trace_rec* trace;
    long long trace_cap;
    signed char* plog;     // LLP_TIMING: phase run by step launch k (-1 none, 0 PRE, 1 MAIN)
    long long plog_cap;
    long long max_rounds;
    SchedParams sp;
};

__device__ __forceinline__ ListRef cl_of(const GArgs& a, int r) { return (r & 1) ? a.cl1 : a.cl0; }

// --------------------------------------------------------------- init
__global__ void k_graph_init(GArgs a, const int* warm) {
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < a.n; v += nt) {
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
    for (long long s = tid; s < a.nseg; s += nt) {
        a.cl0.seg[s] = 0ull;
        a.cl1.seg[s] = 0ull;
        a.wl.seg[s] = 0ull;
        a.cl0.segmin[s] = LLP_INF;
        a.cl1.segmin[s] = LLP_INF;
    }
    if (blockIdx.x == 0) {
        // delta base width: 2^floor(log2 of the mean weight of a stride sample of
        // the in-arcs) (1 for unit weights)
        __shared__ long long wsum[4];
        long long sum = 0;
        int cnt = 0;
        if (!a.unit_w && !a.jobs && a.in_w && a.m > 0) {
            for (int i = threadIdx.x; i < 4096; i += blockDim.x) {
                long long e = (long long)i * a.m / 4096;
                sum += a.in_w[e];
            }
            cnt = 4096;
        }
        sum = wave_sum64(sum);
        if (lane() == 0) wsum[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long t = 0;
            for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wsum[k];
            int base = 1;
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
struct GShared {
    int cnt[MAX_SEG];
    int epre[MAX_SEG + 1];
    int own[GW][64];
    unsigned long long ctr;    // appends to the phase's main output list
    unsigned long long cctr;   // PRE in pull rounds: entries carried into CL[r]
    int cmin;                  // smallest distance appended to CL[r] by this workgroup
    int tot_edges, tot_count;
    int code;
    int tmp1;
    int carried;
    int tmp[GW + 1];
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

// Push: single-arc partial advance of each out-neighbour (Definition 3).
__device__ __forceinline__ void push_body(const GArgs& a, const EdgeCtx& c, int r, const ListRef& out,
                                          GShared& sh, bool& ovf, long long& nadv, bool skip) {
    int umine = c.mine_valid ? guard(c.mine.x, a.n, a.ctrl->diag, 61) : 0;
    int gmine = c.mine_valid ? a.G[umine] : 0;
    int dmine = (c.mine_valid && a.jobs) ? a.vdur[umine] : 0;
    int gu = shfl(gmine, c.j);
    int du = shfl(dmine, c.j);
    bool changed = false, advanced = false;
    int x = 0, ob = 0, od = 0, cand = 0;
    if (c.active && !skip) {
        int e = guard(c.csr, a.m, a.ctrl->diag, 62, c.own.y, c.own.z);
        x = guard(a.out_dst[e], a.n, a.ctrl->diag, 63);
        if (a.jobs) {
            cand = jobs_cand(gu, du, ovf);
        } else {
            int w = a.unit_w ? 1 : a.out_w[e];
            cand = pull_cand(gu, w, ovf);
        }
        if (cand > 0 && cand > a.G[x]) {
            int old = amax(&a.G[x], cand);
            advanced = old < cand;
            if (advanced) {
                ob = a.out_ptr[x];
                int oe = a.out_ptr[x + 1];
                changed = (amax(&a.cstamp[x], r) < r);
                od = oe - ob;
            }
        }
    }
    if (changed) nadv++;
    append(changed && od > 0, x, ob, od, &sh.ctr, out, &a.ctrl->status);
    if (out.segmin) wave_min_to_lds(advanced, dist_key(a, cand), &sh.cmin);
}

__device__ __forceinline__ void wave_range(int total, int& wb, int& we) {
    const long long W = (long long)gridDim.x * GW;
    const long long w = (long long)blockIdx.x * GW + (threadIdx.x >> 6);
    wb = (int)((long long)total * w / W);
    we = (int)((long long)total * (w + 1) / W);
}

__device__ __forceinline__ void publish(const ListRef& out, unsigned long long ctr, int cmin) {
    out.seg[blockIdx.x] = ctr;
    if (out.segmin) out.segmin[blockIdx.x] = cmin;
}

// Delta width of a round code (0: no buckets).
__device__ __forceinline__ int delta_of(const GArgs& a, int code) {
    const int mode = code & 3, dc = (code >> 8) & 3;
    if (a.jobs || mode == MODE_DENSE) return 0;
    const int base = a.ctrl->dbase > 0 ? a.ctrl->dbase : 1;
    switch (dc) {
        case DCLS_BASE: return base;
        case DCLS_WIDE: return base <= (1 << 27) ? base * 8 : (1 << 30);
        case DCLS_EXPLICIT: return a.sp.delta;
        default: return 0;
    }
}

// --------------------------------------------------------------- PRE
// Round r, first phase: consume CL[r-1], decide the round's code, then
// expand into WL (pull), push (CL[r]) or nothing (dense).  k: step launch.
__device__ void pre_phase(const GArgs& a, int r, int k, GShared& sh) {
    const ListRef in = cl_of(a, r - 1);
    const ListRef out = cl_of(a, r);
    load_segments(in.seg, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);
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
        }
        return;
    }
    if ((long long)r > a.max_rounds) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.ctrl->over = 1;
            a.ctrl->done = 1;
            a.ctrl->last_round = r - 1;
        }
        return;
    }
    // schedule decision (identical in every workgroup)
    if (threadIdx.x < 64) {
        int code = decide_mode(a.sp, a.ctrl->hist[(r + 1) & 1], r, sh.tot_count, sh.tot_edges, a.n, a.m,
                               force_dense);
        if (threadIdx.x == 0) sh.code = code;
    }
    if (threadIdx.x == 0) {
        sh.ctr = 0ull;
        sh.cctr = 0ull;
        sh.cmin = LLP_INF;
        sh.carried = 0;
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        GCtrl* c = a.ctrl;
        c->mode = code;
        c->rounds = r;
        // the next step launch: MAIN of this round, or PRE of the next one after a push
        c->step_phase[(k + 1) & 1] = mode == MODE_PUSH ? 0 : 1;
        c->step_round[(k + 1) & 1] = r;
        if (a.plog && k < a.plog_cap) a.plog[k] = 0;
        c->adv += sh.tot_count;
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
            a.trace[r - 1] = t;
        }
    }
    if (mode == MODE_DENSE) return;
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
        for_edges(src, wb, we, own, [&](const EdgeCtx& c) {
            bool skip = carry_step(a, c, r, hi, out, &sh.ctr, sh);
            push_body(a, c, r, out, sh, ovf, nadv, skip);
        });
        __syncthreads();
        if (threadIdx.x == 0) publish(out, sh.ctr, sh.cmin);
    }
    if (threadIdx.x == 0 && sh.carried) atomicAdd(&a.ctrl->carried[r & 1], sh.carried);
    if (__any(ovf) && lane() == 0) st_relaxed(&a.ctrl->ovf, 1);
}

// --------------------------------------------------------------- MAIN
// Round r, second phase (pull and dense rounds): evaluate WL (or every
// vertex) and produce CL[r].  verify != 0: a dense round on the final state
// that must change nothing.
__device__ void main_phase(const GArgs& a, int r, int verify, int k, GShared& sh) {
    const int code = verify ? MODE_DENSE : a.ctrl->mode;
    const int mode = code & 3;
    if (!verify && blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctrl->step_phase[(k + 1) & 1] = 0;
        a.ctrl->step_round[(k + 1) & 1] = r;
        if (a.plog && k < a.plog_cap) a.plog[k] = 1;
    }
    if (mode == MODE_PUSH) return;
    const ListRef out = verify ? a.wl : cl_of(a, r);   // verify writes into WL's storage
    if (threadIdx.x == 0) {
        // pull rounds continue the segment PRE started with carried entries
        const bool cont = mode == MODE_PULL && !verify;
        sh.ctr = cont ? out.seg[blockIdx.x] : 0ull;
        sh.cmin = (cont && out.segmin) ? out.segmin[blockIdx.x] : LLP_INF;
    }
    int* own = sh.own[threadIdx.x >> 6];
    bool ovf = false;
    long long nadv = 0;
    int wb, we;
    if (mode == MODE_DENSE) {
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0 && !verify) {
            a.ctrl->cand += a.n;
            a.ctrl->edges += a.m;
        }
        int rr = verify ? r + 1 : r;
        DenseSrc src{a.in_ptr, a.n, a.ctrl->diag, 0};
        wave_range(a.m, wb, we);
        for_edges(src, wb, we, own,
                  [&](const EdgeCtx& c) { eval_body(a, c, rr, out, sh, ovf, nadv); });
    } else {
        load_segments(a.wl.seg, a.nseg, sh.cnt, sh.epre, sh.tmp, &sh.tot_edges, &sh.tot_count);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            a.ctrl->cand += sh.tot_count;
            a.ctrl->edges += sh.tot_edges;
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
// slot k & 1 (PRE of the next round, or MAIN of the current one), so a push
// round costs one launch and a pull or dense round two.  The slots
// alternate, so no workgroup of launch k reads the slot launch k writes.
__global__ void __launch_bounds__(GB) k_graph_step(GArgs a, int k) {
    __shared__ GShared sh;
    if (ld_relaxed(&a.ctrl->done) || ld_relaxed(&a.ctrl->status)) return;
    const int ph = a.ctrl->step_phase[k & 1];
    const int rr = a.ctrl->step_round[k & 1];
    if (ph == 0) pre_phase(a, rr + 1, k, sh);
    else main_phase(a, rr, 0, k, sh);
}

__global__ void __launch_bounds__(GB) k_graph_verify(GArgs a, int r) {
    __shared__ GShared sh;
    main_phase(a, r, 1, 0, sh);
}

// --------------------------------------------------------------- finish
// Overflow: a vertex still at the bottom with a reached in-neighbour has a
// true distance >= INF.  Only run when a candidate overflowed.
// Jobs: every completion time S[j] + dur[j] must fit int32 (always checked).
__global__ void k_graph_ovf(GArgs a) {
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

// In place: G -> distance (INF for unreached).
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
    return graph_ws(n, m, graph_wgs_per_cu(chunk), nullptr, nullptr, 0);
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

static int launch_grid_1d(int64_t work) {
    int64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    int cap = device_info().cus * 8;
    return (int)(g < cap ? g : cap);
}

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
    int s = sched_params(o, bfs || jobs_dur || g->out_w != nullptr, &a.sp);
    if (s) return s;

    const int per_cu = graph_wgs_per_cu(o.chunk);
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
    // step launches: at most two per round; the batch doubles up to 32
    const int64_t max_launches = 2 * max_rounds + 4;
    int64_t k = 0;
    int batch = 8;
    int status = LLP_OK;
    std::vector<hipEvent_t> evs;     // LLP_TIMING: one pair around each step launch
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
                hipLaunchKernelGGL(k_graph_step, dim3(a.nseg), dim3(GB), 0, st, a, (int)k);
                LLP_HIP(hipEventRecord(e1, st));
                evs.push_back(e0);
                evs.push_back(e1);
            } else {
                hipLaunchKernelGGL(k_graph_step, dim3(a.nseg), dim3(GB), 0, st, a, (int)k);
            }
        }
        LLP_HIP(hipGetLastError());
        s = readback(st, a.ctrl, &h, sizeof(h));
        if (s) return s;
        if (h.status) break;
        if (h.done) {
            if (h.over) status = LLP_E_NOT_CONVERGED;
            break;
        }
        if (o.abort_host && *o.abort_host) { status = LLP_E_ABORTED; break; }
        if (k >= max_launches) { status = LLP_E_NOT_CONVERGED; break; }
        if (batch < 32) batch *= 2;
    }
    if (status == LLP_OK && h.status == 0 && (o.flags & LLP_VERIFY)) {
        hipLaunchKernelGGL(k_graph_verify, dim3(a.nseg), dim3(GB), 0, st, a, (int)h.last_round + 1);
    }
    if (h.status == 0) hipLaunchKernelGGL(k_graph_ovf, dim3(g1), dim3(256), 0, st, a);
    if (!jobs_dur) hipLaunchKernelGGL(k_graph_decode, dim3(launch_grid_1d(g->n)), dim3(256), 0, st, out, g->n);
    LLP_HIP(hipGetLastError());
    if (timing) LLP_HIP(hipEventRecord(ev1, st));
    s = readback(st, a.ctrl, &h, sizeof(h));
    if (s) return s;
    if (o.stats) {
        memset(o.stats, 0, sizeof(*o.stats));
        o.stats->rounds = h.rounds;
        o.stats->candidates = h.cand;
        o.stats->edges_inspected = h.edges;
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
            o.stats->pre_ms = pms;
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

}  // namespace llp

extern "C" {

int llp_solve_sssp(const llp_graph* g, int32_t source, int32_t* dist, const llp_opts* opts) {
    return llp::solve_graph(g, source, dist, opts, false);
}

int llp_solve_bfs(const llp_graph* g, int32_t source, int32_t* level, const llp_opts* opts) {
    return llp::solve_graph(g, source, level, opts, true);
}

}  // extern "C"
