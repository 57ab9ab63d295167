// llp_dev.h - device building blocks shared by the LLP sweep kernels (gfx950,
// wave64).  Wave-level scans and reductions, ballot compaction, atomic
// helpers, and the edge-balanced list iterator used by every graph phase.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define LLP_WAVE 64
#define LLP_INF 2147483647

namespace llp {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of mask strictly below this lane
__device__ __forceinline__ int mbcnt(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int shfl(int v, int src) { return __shfl(v, src, LLP_WAVE); }

// Wave scans by DPP (all 64 lanes active): four row shifts give the
// inclusive scan within each row of 16 lanes, then the last lane of row 0
// is broadcast into row 1 and that of row 2 into row 3, and lane 31 (rows 0
// and 1 complete) into rows 2 and 3.  A lane whose source lies outside its
// row, or whose row the mask leaves out, takes the identity.  No lane
// comparison or LDS crossbar trip is involved.
constexpr int DPP_ROW_SHR = 0x110;     // + shift (1..15)
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR + 1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR + 2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR + 4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR + 8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST31, 0xc, 0xf, false);
    return x;
}

__device__ __forceinline__ long long wave_incl_sum64(long long x) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < LLP_WAVE; d <<= 1) {
        long long y = __shfl_up(x, d, LLP_WAVE);
        if (l >= d) x += y;
    }
    return x;
}

// inclusive max scan over the wave (same steps as wave_incl_sum)
__device__ __forceinline__ int wave_incl_max(int x) {
    constexpr int lo = -2147483647 - 1;
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_SHR + 1, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_SHR + 2, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_SHR + 4, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_SHR + 8, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_BCAST15, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(lo, x, DPP_ROW_BCAST31, 0xc, 0xf, false));
    return x;
}

// maximum over the wave, in every lane: the DPP max scan, whose lane 63
// holds the whole wave's maximum, then one shuffle from that lane
__device__ __forceinline__ int wave_max(int x) {
    return __shfl(wave_incl_max(x), 63, LLP_WAVE);
}

__device__ __forceinline__ long long wave_sum64(long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, LLP_WAVE);
    return x;
}

// Segmented inclusive max scan: lanes with equal seg (contiguous runs) are
// reduced together; the last lane of each run ends with the run maximum.
__device__ __forceinline__ int seg_incl_max(int x, int seg) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < LLP_WAVE; d <<= 1) {
        int y = __shfl_up(x, d, LLP_WAVE);
        int s = __shfl_up(seg, d, LLP_WAVE);
        if (l >= d && s == seg) x = max(x, y);
    }
    return x;
}

// Index guards.  An index outside [0, bound) is replaced by 0, so neither a
// malformed input nor an inconsistent list can turn into an out-of-bounds
// access.  clampi() only marks `bad` (the phase then reports LLP_E_INPUT);
// guard() also records the first offending site and values in `diag`
// (diag[0] = site id, diag[1..4] = index, bound, two context values).
__device__ __forceinline__ int clampi(int i, int bound, bool& bad) {
    bool ok = (unsigned)i < (unsigned)bound;
    bad |= !ok;
    return ok ? i : 0;
}

__device__ __noinline__ void record_diag(int* diag, int site, int i, int bound, int c0, int c1) {
    int expected = 0;
    if (__hip_atomic_compare_exchange_strong(diag, &expected, site, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
        diag[1] = i;
        diag[2] = bound;
        diag[3] = c0;
        diag[4] = c1;
    }
}

__device__ __forceinline__ int guard(int i, int bound, int* diag, int site, int c0 = 0, int c1 = 0) {
    bool ok = (unsigned)i < (unsigned)bound;
    if (__builtin_expect(!ok, 0)) {
        if (diag) record_diag(diag, site, i, bound, c0, c1);
        return 0;
    }
    return i;
}

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ int amax(int* p, int v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int amin(int* p, int v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int aadd(int* p, int v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned aor(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// set the device status word to s if it is still 0 (first error wins)
__device__ __forceinline__ void set_status(int* status, int s) {
    int expected = 0;
    __hip_atomic_compare_exchange_strong(status, &expected, s, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace llp
