// llp_sched.h - per-round schedule choice of the graph sweep.
//
// The paper leaves the choice of solver (all-indices, worklist, buckets) to
// the user per workload and names a runtime monitor that samples the
// frontier and switches policy as future work (Section 6, Section 7).  Every
// choice here is only a schedule: the least fixpoint is the same whatever
// the mode of each round.  Modes: pull over the compacted candidate
// worklist, dense pull over every index, push along out-arcs.
//
// LLP_SCHED_LEARNED runs a 12 -> 64 -> 64 -> 5 MLP (bf16 weights, fp32
// accumulation) on 12 frontier features in one wave of every workgroup; all
// workgroups compute bit-identical inputs and therefore the same decision.
#pragma once

#include "llp_dev.h"
#include "../../include/llp.h"

namespace llp {

struct SchedHist {
    int r;               // round that wrote this record
    int mode;            // mode of that round
    int cl_count;        // changed indices that round consumed (input list)
    int cl_edges;
    int wl_count;        // candidates it evaluated (pull rounds)
    int wl_edges;
    int pad0, pad1;
    long long adv_total; // cumulative changed indices
};

struct SchedParams {
    unsigned sched;
    unsigned flags;
    int delta;
    int can_push;
    unsigned long long seed;
    const unsigned short* mlp;   // bf16 parameter block (LLP_MLP_PARAMS), device
    float dense_frac;            // HYBRID: dense when changed out-arcs exceed this fraction of m, else push
    int push_dclass;             // HYBRID: delta class of its push rounds (DCLS_WIDE on sparse weighted
                                 // graphs, DCLS_NONE otherwise)
    const int* plan;             // SCRIPT: round codes (device)
    long long plan_len;
};

enum { DCLS_BASE = 0, DCLS_WIDE = 1, DCLS_NONE = 2, DCLS_EXPLICIT = 3 };

// LLP_SCHED_LEARNED consults the network on rounds of at least m / this many
// frontier arcs
constexpr int LEARNED_MIN_FRAC = 256;

__device__ __forceinline__ int round_code(int mode, int dcls) { return mode | (dcls << 8); }

int sched_params(const llp_opts& o, bool can_push, SchedParams* sp);
const unsigned short* learned_weights_device();
// The frontier-width hybrid's parameters for a problem (kind LLP_KIND_SSSP,
// LLP_KIND_BFS or LLP_KIND_JOBS) of n indices and m arcs: dense above a
// fraction of the arcs (SSSP 1/3, BFS 1/14, jobs 1/2), push otherwise, with
// wide delta buckets on weighted graphs of 2 to 8 arcs per vertex.
void hybrid_params(int kind, long long n, long long m, bool can_push, SchedParams* sp);

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float(((unsigned)h) << 16);
}
// round to nearest even
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
    unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float round_bf16(float f) { return bf16_to_f32(f32_to_bf16(f)); }

// Round code of the frontier-width hybrid for a round whose input list has
// cl_edges out-arcs.
__device__ __forceinline__ int hybrid_code(const SchedParams& sp, int cl_edges, int m) {
    if ((float)cl_edges > sp.dense_frac * (float)m) return round_code(1, DCLS_NONE);
    return sp.can_push ? round_code(2, sp.push_dclass) : round_code(0, DCLS_NONE);
}

// The 12 round features (all lanes compute the same values).  hyb: the
// hybrid's round code for this round (the threshold signal the network may
// follow or overrule).
__device__ __forceinline__ void round_features(float f[12], int r, int cl_count, int cl_edges, int n, int m,
                                               const SchedHist& h, int hyb) {
    const float ln = __log2f(1.0f + (float)n), lm = __log2f(1.0f + (float)m);
    const float davg = (float)m / (float)(n > 0 ? n : 1);
    f[0] = __log2f(1.0f + (float)cl_count) / ln;
    f[1] = __log2f(1.0f + (float)cl_edges) / (lm > 0.f ? lm : 1.f);
    f[2] = (float)cl_count / (float)n;
    f[3] = m > 0 ? (float)cl_edges / (float)m : 0.f;
    f[4] = (cl_count > 0 ? (float)cl_edges / (float)cl_count : 0.f) / (davg > 0.f ? davg : 1.f);
    // the hybrid's choice: 0 push, 0.5 push with wide buckets, 0.25 pull, 1 dense
    const int hm = hyb & 3;
    f[5] = hm == 1 ? 1.f : (hm == 0 ? 0.25f : (((hyb >> 8) & 3) == DCLS_WIDE ? 0.5f : 0.f));
    f[6] = __log2f(1.0f + davg) / 8.f;
    f[7] = __log2f(1.0f + (float)cl_count) - __log2f(1.0f + (float)h.cl_count);
    f[8] = h.mode == 2 ? 1.f : 0.f;
    f[9] = h.mode == 1 ? 1.f : 0.f;
    f[10] = (float)r / (float)(r + 16);
    f[11] = (float)h.adv_total / (float)n;
    for (int i = 0; i < 12; ++i) f[i] = round_bf16(f[i]);
}

__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// Lane j's weights of the network: its rows of W1 (24 B) and W2 (128 B),
// column j of W3 and its two biases, read with wide loads.  Loaded before the
// round's list totals are scanned, so their latency overlaps that scan.
struct MlpLane {
    uint2 w1[3];
    uint4 w2[8];
    float w3[5];
    float b1, b2;
};

__device__ __forceinline__ MlpLane mlp_load(const unsigned short* P) {
    const int j = lane();
    const unsigned short* W1 = P;
    const unsigned short* b1 = W1 + 64 * 12;
    const unsigned short* W2 = b1 + 64;
    const unsigned short* b2 = W2 + 64 * 64;
    const unsigned short* W3 = b2 + 64;
    MlpLane w;
    // W1 row j starts at 24 j bytes (8-byte aligned), W2 row j at 1664 + 128 j
    const uint2* r1 = reinterpret_cast<const uint2*>(W1 + j * 12);
    const uint4* r2 = reinterpret_cast<const uint4*>(W2 + j * 64);
#pragma unroll
    for (int q = 0; q < 3; ++q) w.w1[q] = r1[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) w.w2[q] = r2[q];
#pragma unroll
    for (int o = 0; o < 5; ++o) w.w3[o] = bf16_to_f32(W3[o * 64 + j]);
    w.b1 = bf16_to_f32(b1[j]);
    w.b2 = bf16_to_f32(b2[j]);
    return w;
}

// Wave-level MLP forward: out[5] logits in every lane.  Lane j holds hidden
// unit j of both layers; the first layer's activations are broadcast from
// LDS (h[64], private to the calling wave).  Products are summed in input
// order, one at a time.
__device__ inline void mlp_forward_wave(const unsigned short* P, const MlpLane& w, const float f[12], float out[5],
                                        float* h) {
    const int j = lane();
    const unsigned short* b3 = P + 64 * 12 + 64 + 64 * 64 + 64 + 5 * 64;
    const unsigned u1[6] = {w.w1[0].x, w.w1[0].y, w.w1[1].x, w.w1[1].y, w.w1[2].x, w.w1[2].y};
    float a = w.b1;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        a += bf16_lo(u1[k]) * f[2 * k];
        a += bf16_hi(u1[k]) * f[2 * k + 1];
    }
    h[j] = round_bf16(fmaxf(a, 0.f));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float a2 = w.b2;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned u[4] = {w.w2[q].x, w.w2[q].y, w.w2[q].z, w.w2[q].w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a2 += bf16_lo(u[t]) * h[8 * q + 2 * t];
            a2 += bf16_hi(u[t]) * h[8 * q + 2 * t + 1];
        }
    }
    float h2 = round_bf16(fmaxf(a2, 0.f));
    for (int o = 0; o < 5; ++o) {
        float t = w.w3[o] * h2;
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        out[o] = t + bf16_to_f32(b3[o]);
    }
}

__device__ __forceinline__ unsigned long long mix64d(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Code of round r: mode (bits 0-1: 0 pull over the worklist, 1 dense pull,
// 2 push) and delta class (bits 8-9).  Call from a whole wave; the result is
// wave-uniform, and identical in every workgroup (same inputs).
__device__ inline int decide_mode(const SchedParams& sp, const SchedHist& h, int r, int cl_count, int cl_edges,
                                  int n, int m, int force_dense, const MlpLane& wl, float* lds64) {
    if (force_dense) return round_code(1, DCLS_NONE);
    switch (sp.sched) {
        case LLP_SCHED_FIXED: {
            const int dc = sp.delta > 0 ? DCLS_EXPLICIT : DCLS_NONE;
            if (sp.flags & LLP_DENSE) return round_code(1, dc);
            if ((sp.flags & LLP_PUSH) && sp.can_push) return round_code(2, dc);
            return round_code(0, dc);
        }
        case LLP_SCHED_HYBRID:
            return hybrid_code(sp, cl_edges, m);
        case LLP_SCHED_RANDOM: {
            unsigned long long z = mix64d(sp.seed * 0x9E3779B97F4A7C15ull + (unsigned long long)r);
            int k = (int)(z % (unsigned long long)(sp.can_push ? 3 : 2));
            int dc = (int)((z >> 32) % 3ull);
            return round_code(k, dc);
        }
        case LLP_SCHED_SCRIPT: {
            if (!sp.plan || (long long)r > sp.plan_len) return round_code(0, DCLS_NONE);
            int c = sp.plan[r - 1];
            int mode = c & 3, dc = (c >> 8) & 3;
            if (mode == 3) return hybrid_code(sp, cl_edges, m);   // the hybrid decides this round
            if (mode == 2 && !sp.can_push) mode = 0;
            if (dc == DCLS_EXPLICIT && sp.delta <= 0) dc = DCLS_NONE;
            return round_code(mode, dc);
        }
        case LLP_SCHED_LEARNED: {
            if (!sp.mlp) return round_code(0, DCLS_NONE);
            // the network costs about 1.8 us per round; on rounds of fewer than
            // m / 256 frontier arcs no decision can gain that back, and the
            // hybrid's code is taken
            if ((long long)cl_edges * LEARNED_MIN_FRAC < (long long)m) return hybrid_code(sp, cl_edges, m);
            float f[12], o[5];
            round_features(f, r, cl_count, cl_edges, n, m, h, hybrid_code(sp, cl_edges, m));
            mlp_forward_wave(sp.mlp, wl, f, o, lds64);
            int dc = DCLS_BASE;
            if (o[3] > o[2]) dc = DCLS_WIDE;
            if (o[4] > fmaxf(o[2], o[3])) dc = DCLS_NONE;
            if (o[0] > 0.f && sp.can_push) return round_code(2, dc);
            if (o[1] > 0.f) return round_code(1, dc);
            return round_code(0, dc);
        }
        default:
            return round_code(0, DCLS_NONE);
    }
}

// Record round r's input list in the history slot for the next decision.
__device__ __forceinline__ void hist_push(SchedHist& dst, const SchedHist& prev, int r, int mode, int cl_count,
                                          int cl_edges) {
    dst.r = r;
    dst.mode = mode;
    dst.cl_count = cl_count;
    dst.cl_edges = cl_edges;
    dst.wl_count = 0;
    dst.wl_edges = 0;
    dst.adv_total = prev.adv_total + cl_count;
}

}  // namespace llp
