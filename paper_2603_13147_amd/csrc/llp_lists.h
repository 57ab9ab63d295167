// llp_lists.h - worklists of the LLP sweep and the edge-balanced iterator.
//
// A list is produced by one kernel and consumed by the next.  Each producing
// workgroup owns a private segment of `cap` entries and reserves slots with a
// packed 64-bit LDS atomic (count | edges << 32), so a list is built without
// any contended global counter; at kernel end the workgroup publishes its
// packed total in seg[blockIdx.x].  An entry is {v, rb, off, deg}: the index,
// the first CSR position of its row, its offset in the segment's virtual edge
// space and its row length.  Entries with deg == 0 are never stored.
//
// A consumer scans the seg[] totals in LDS (one pass per workgroup), splits
// the list's total edge count evenly over all waves and walks each wave's
// range 64 edges at a time: a window of up to 64 entries is loaded, each edge
// lane finds its owning entry by an LDS scatter of entry start positions and
// a max-scan, and the phase body sees (owner lane, owner index, CSR position).
// The dense source treats every index 0..n-1 as an entry of a CSR row.
#pragma once

#include "llp_dev.h"

namespace llp {

// List words read or written by workgroups of the same launch (the
// multi-round tail kernel) go through agent-scope atomics, which bypass the
// caches that are not coherent between compute units; lists that only cross
// a launch boundary use plain accesses (COH = false).
template <bool COH>
__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long* p) {
    if constexpr (COH) return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH>
__device__ __forceinline__ void st_u64(unsigned long long* p, unsigned long long v) {
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ int ld_i32(const int* p) {
    if constexpr (COH) return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH>
__device__ __forceinline__ void st_i32(int* p, int v) {
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool COH>
__device__ __forceinline__ int4 ld_ent(const int4* p) {
    if constexpr (COH) {
        const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
        const unsigned long long a = ld_u64<true>(q), b = ld_u64<true>(q + 1);
        return make_int4((int)(unsigned)a, (int)(unsigned)(a >> 32), (int)(unsigned)b, (int)(unsigned)(b >> 32));
    } else {
        return *p;
    }
}
template <bool COH>
__device__ __forceinline__ void st_ent(int4* p, int4 v) {
    if constexpr (COH) {
        unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
        st_u64<true>(q, (unsigned long long)(unsigned)v.x | ((unsigned long long)(unsigned)v.y << 32));
        st_u64<true>(q + 1, (unsigned long long)(unsigned)v.z | ((unsigned long long)(unsigned)v.w << 32));
    } else {
        *p = v;
    }
}

struct ListRef {
    int4* ent;                    // nb * cap entries
    unsigned long long* seg;      // nb packed totals
    int* segmin;                  // nb per-segment minimum key (nullable; graph lists: decoded distance)
    int cap;
};

// Per-workgroup view of a consumed list: segment counts and edge prefix in LDS.
struct SegView {
    const int4* ent;
    int cap;
    int nseg;
    const int* cnt;     // [nseg] (LDS)
    const int* epre;    // [nseg + 1] exclusive edge prefix (LDS)
    int total_edges;
    int total_count;
};

// This thread's packed segment totals (segments t * per .. t * per + per - 1,
// per = ceil(nseg / blockDim) <= 8), fetched ahead of the scan so that a
// kernel can issue them together with its other first loads.
struct SegRegs {
    unsigned long long x[8];
};
template <bool COH = false>
__device__ inline void seg_fetch(const unsigned long long* seg, int nseg, SegRegs& s) {
    const int per = (nseg + blockDim.x - 1) / blockDim.x;
    const int b = threadIdx.x * per, e = min(b + per, nseg);
#pragma unroll
    for (int k = 0; k < 8; ++k) s.x[k] = (k < per && b + k < e) ? ld_u64<COH>(seg + b + k) : 0ull;
}

// Block-wide scan of fetched segment totals into LDS arrays.
// lds_cnt[nseg], lds_epre[nseg+1] must be __shared__ buffers.  (A template,
// like every helper here that declares its own LDS.)
template <int = 0>
__device__ inline void seg_scan(const SegRegs& s, int nseg, int* lds_cnt, int* lds_epre,
                                int* lds_tmp /* >= blockDim/64 + 1 ints */, int* tot_edges, int* tot_count) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int per = (nseg + nt - 1) / nt;   // <= 8 (nseg <= 2048, >= 256 threads)
    const int b = t * per, e = min(b + per, nseg);
    int se = 0, sc = 0;
    int eds[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = b + k;
        eds[k] = 0;
        if (k < per && i < e) {
            const unsigned long long x = s.x[k];
            int c = (int)(x & 0xffffffffull), ed = (int)(x >> 32);
            lds_cnt[i] = c;
            eds[k] = ed;
            sc += c;
            se += ed;
        }
    }
    // block exclusive scan of se (edges) and total of sc (counts)
    int w = t >> 6, l = lane();
    int incl = wave_incl_sum(se);
    long long csum = wave_sum64(sc);
    __shared__ int wsum[16];
    __shared__ long long wcnt[16];
    if (l == 63) wsum[w] = incl;
    if (l == 0) wcnt[w] = csum;
    __syncthreads();
    int nw = nt >> 6;
    int woff = 0;
    long long ctot = 0;
    int etot = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < w) woff += wsum[k];
        etot += wsum[k];
        ctot += wcnt[k];
    }
    int run = woff + incl - se;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int i = b + k;
        if (k < per && i < e) {
            lds_epre[i] = run;
            run += eds[k];
        }
    }
    if (t == 0) lds_epre[nseg] = etot;
    *tot_edges = etot;
    *tot_count = (int)ctot;
    (void)lds_tmp;
    __syncthreads();
}

// Fetch and scan in one step.
template <bool COH = false>
__device__ inline void load_segments(const unsigned long long* seg, int nseg, int* lds_cnt, int* lds_epre,
                                     int* lds_tmp /* >= blockDim/64 + 1 ints */, int* tot_edges, int* tot_count) {
    SegRegs s;
    seg_fetch<COH>(seg, nseg, s);
    seg_scan(s, nseg, lds_cnt, lds_epre, lds_tmp, tot_edges, tot_count);
}

// ---------------------------------------------------------------- sources
// Cursor: (seg, idx) for lists; (v, -) for the dense source.
struct Cursor {
    int s;
    int i;
};

// Dense: every index v with row [ptr[v], ptr[v+1]).
struct DenseSrc {
    const int* ptr;
    int n;          // rows
    int* diag;

    // largest v with ptr[v] <= e (e < ptr[n]); 64-ary search, wave-uniform result
    __device__ Cursor locate(int e) const {
        int lo = 0, hi = n;  // answer in [lo, hi)
        while (hi - lo > 64) {
            int step = (hi - lo + 63) / 64;
            int probe = lo + lane() * step;
            bool ok = probe < hi && ptr[guard(probe, n + 1, diag, 11, lo, hi)] <= e;
            int c = __popcll(ballot(ok));
            lo = lo + (c - 1) * step;
            hi = min(lo + step, hi);
        }
        int probe = lo + lane();
        bool ok = probe < hi && ptr[guard(probe, n + 1, diag, 12, lo, hi)] <= e;
        int c = __popcll(ballot(ok));
        return Cursor{guard(lo + c - 1, n, diag, 13, e, c), 0};
    }
    __device__ int avail(const Cursor& c) const { return n - c.s; }
    __device__ int4 load(const Cursor& c, int l) const {
        int v = c.s + l;
        int vv = guard(v, n, diag, 14, c.s, l);
        int b = ptr[vv];
        return make_int4(v, b, b, ptr[vv + 1] - b);
    }
    __device__ Cursor advance(Cursor c, int k) const { c.s += k; return c; }
};

// Segmented list.
template <bool COH = false>
struct ListSrcT {
    SegView sv;
    int* diag;

    __device__ Cursor locate(int e) const {
        // segment: largest s with epre[s] <= e and cnt[s] > 0
        int lo = 0, hi = sv.nseg;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (sv.epre[mid] <= e) lo = mid; else hi = mid;
        }
        int s = lo;
        while (s < sv.nseg - 1 && sv.cnt[s] == 0) ++s;   // empty segments have epre[s] == epre[s+1]
        int local = e - sv.epre[s];
        const int4* base = sv.ent + (long long)s * sv.cap;
        int lo2 = 0, hi2 = min(sv.cnt[s], sv.cap);
        while (hi2 - lo2 > 64) {
            int step = (hi2 - lo2 + 63) / 64;
            int probe = lo2 + lane() * step;
            bool ok = probe < hi2 && ld_ent<COH>(base + guard(probe, sv.cap, diag, 21, lo2, hi2)).z <= local;
            int c = __popcll(ballot(ok));
            lo2 = lo2 + (c - 1) * step;
            hi2 = min(lo2 + step, hi2);
        }
        int probe = lo2 + lane();
        bool ok = probe < hi2 && ld_ent<COH>(base + guard(probe, sv.cap, diag, 22, lo2, hi2)).z <= local;
        int c = __popcll(ballot(ok));
        return Cursor{s, guard(lo2 + c - 1, sv.cap, diag, 23, e, local)};
    }
    __device__ int avail(const Cursor& c) const { return c.s < sv.nseg ? min(sv.cnt[c.s], sv.cap) - c.i : 0; }
    __device__ int4 load(const Cursor& c, int l) const {
        int s = guard(c.s, sv.nseg, diag, 24, c.i, l);
        int i = guard(c.i + l, sv.cap, diag, 25, c.s, l);
        int4 x = ld_ent<COH>(sv.ent + (long long)s * sv.cap + i);
        x.z += sv.epre[s];
        return x;
    }
    __device__ Cursor advance(Cursor c, int k) const {
        c.i += k;
        if (c.s < sv.nseg && c.i >= min(sv.cnt[c.s], sv.cap)) {
            // past this segment: jump to the one holding the next edge, the
            // last segment whose edge prefix is at most that edge's index
            // (every entry has arcs, so the empty segments in between share
            // its prefix).  A narrow list leaves most segments empty, and
            // stepping over them one at a time cost the wave that finished
            // the list several microseconds per round.
            const int e = sv.epre[c.s + 1];
            int lo = c.s + 1, hi = sv.nseg;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sv.epre[mid] <= e) lo = mid; else hi = mid;
            }
            c.s = lo;
            c.i = 0;
            // no edge after this segment: the trailing segments are empty
            if (c.s < sv.nseg && min(sv.cnt[c.s], sv.cap) == 0) c.s = sv.nseg;
        }
        return c;
    }
};

using ListSrc = ListSrcT<false>;

// Edge-lane context handed to a phase body.
struct EdgeCtx {
    bool active;   // this lane holds an edge of the current iteration
    int j;         // owner lane within the window
    int4 own;      // owner entry {v, rb, off, deg} (virtual off)
    int csr;       // CSR position of this lane's edge
    int4 mine;     // the window entry held by this lane (valid if lane < avail)
    bool mine_valid;
    int base;      // virtual edge range of this iteration: [base, limit)
    int limit;
};

// Walk virtual edges [wb, we) of src; body(ctx) is called once per iteration
// (wave-uniform call, per-lane data in ctx).  own_lds: 64 ints of LDS private
// to the calling wave.
template <class Src, class Body>
__device__ inline void for_edges(const Src& src, int wb, int we, int* own_lds, Body&& body) {
    if (wb >= we) return;
    const int l = lane();
    Cursor cur = src.locate(wb);
    int base = wb;
    int av = src.avail(cur);
    int4 e = (l < av) ? src.load(cur, l) : make_int4(0, 0, LLP_INF, 0);
    while (base < we) {
        if (av <= 0) {                 // inconsistent list: record and stop this wave
            if (l == 0) record_diag(src.diag, 31, base, we, cur.s, cur.i);
            return;
        }
        const bool valid = l < av;
        int last = (av < 64 ? av : 64) - 1;
        int end_last = shfl(e.z + e.w, last);
        if (end_last <= base) {
            // every row of the window ends at or before base (a run of empty
            // rows of a dense CSR): step over them
            const int skip = __popcll(ballot(valid && e.z + e.w <= base));
            cur = src.advance(cur, skip);
            av = src.avail(cur);
            e = (l < av) ? src.load(cur, l) : make_int4(0, 0, LLP_INF, 0);
            continue;
        }
        int limit = min(min(base + 64, we), end_last);
        own_lds[l] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // position base + p belongs to the last row starting at or before it:
        // rows that start before base (or empty rows at base) vote for slot 0
        int sp = e.z - base;
        if (valid && sp < 64) atomicMax(&own_lds[sp > 0 ? sp : 0], l);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        int j = wave_incl_max(own_lds[l]);
        EdgeCtx c;
        c.active = base + l < limit;
        c.j = j;
        c.own = make_int4(shfl(e.x, j), shfl(e.y, j), shfl(e.z, j), shfl(e.w, j));
        c.csr = c.own.y + (base + l - c.own.z);
        c.mine = e;
        c.mine_valid = valid;
        c.base = base;
        c.limit = limit;
        // the next window is known before the body runs: issue its loads first
        // so they overlap the body's memory traffic
        const int done = __popcll(ballot(valid && e.z + e.w <= limit));
        const Cursor nxt = src.advance(cur, done);
        int nav = 0;
        int4 ne = make_int4(0, 0, LLP_INF, 0);
        if (limit < we) {
            nav = src.avail(nxt);
            if (l < nav) ne = src.load(nxt, l);
        }
        body(c);
        cur = nxt;
        base = limit;
        av = nav;
        e = ne;
    }
}

// Append entries to the calling workgroup's segment of `out`.
// want/entry are per lane; lds_ctr is the workgroup's packed LDS counter.
template <bool COH = false>
__device__ inline void append(bool want, int v, int rb, int deg, unsigned long long* lds_ctr, const ListRef& out,
                              int* status) {
    uint64_t m = ballot(want);
    if (!m) return;
    const int l = lane();
    int k = __popcll(m);
    int r = mbcnt(m);
    int d = want ? deg : 0;
    int incl = wave_incl_sum(d);
    int tot = shfl(incl, 63);
    int leader = __ffsll((long long)m) - 1;
    unsigned long long old = 0;
    if (l == leader) old = atomicAdd(lds_ctr, (unsigned long long)k | ((unsigned long long)(unsigned)tot << 32));
    unsigned lo = (unsigned)__shfl((int)(unsigned)(old & 0xffffffffull), leader, LLP_WAVE);
    unsigned hi = (unsigned)__shfl((int)(unsigned)(old >> 32), leader, LLP_WAVE);
    if (want) {
        int idx = (int)lo + r;
        int off = (int)hi + incl - d;
        if (idx < out.cap) st_ent<COH>(out.ent + (long long)blockIdx.x * out.cap + idx, make_int4(v, rb, off, deg));
        else set_status(status, 7);
    }
}

// Fold val of the lanes with want into the workgroup minimum *lds_min (one
// LDS atomic per wave).
__device__ inline void wave_min_to_lds(bool want, int val, int* lds_min) {
    int x = want ? val : 0x7fffffff;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, LLP_WAVE));
    if (lane() == 0 && x != 0x7fffffff) atomicMin(lds_min, x);
}

// Minimum of seg_min[0..nseg) over the workgroup (every thread gets it).
template <bool COH = false>
__device__ inline int load_segmin(const int* seg_min, int nseg, int* lds_tmp1) {
    int x = 0x7fffffff;
    for (int i = threadIdx.x; i < nseg; i += blockDim.x) x = min(x, ld_i32<COH>(seg_min + i));
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, LLP_WAVE));
    if (threadIdx.x == 0) *lds_tmp1 = 0x7fffffff;
    __syncthreads();
    if (lane() == 0) atomicMin(lds_tmp1, x);
    __syncthreads();
    return *lds_tmp1;
}

}  // namespace llp
