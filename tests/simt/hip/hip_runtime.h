// CPU emulation of the part of the HIP programming interface that libllp's
// graph sweep uses: test infrastructure only.  tests/test_simt_graph.py
// compiles the sweep's own sources (graph.hip and the host code) against this
// header with g++ and AddressSanitizer into a separate test library, so the
// kernels' index arithmetic can be checked on the CPU on inputs that are not
// run on the GPU; libllp.so never includes it.
//
// Each thread of a workgroup is a fiber; wave intrinsics (ballot, shuffles,
// wave barriers) wait until every live lane of the wave has arrived at the
// same one; __syncthreads waits for every live thread of the workgroup.  Lanes
// that reach different wave operations, or a shuffle that reads a lane that
// has finished, abort with a report.  Workgroups of a launch run one after
// another, in index order or (SIMT_SHUFFLE set) a seeded random order.
// "Device" memory is host memory filled with 0xA5 bytes and ending at an
// unmapped page, so a read past the end of any allocation faults at once.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline __attribute__((always_inline))
#define __noinline__ __attribute__((noinline)) inline
#define __launch_bounds__(...)
// every __shared__ variable lives in one section, so that a cooperative
// launch (all workgroups live at once) can give each workgroup its own copy
#define __shared__ __attribute__((section("simt_lds"))) static
#define __align__(x) __attribute__((aligned(x)))

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3s { unsigned x, y, z; };

struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
struct uint4 { unsigned x, y, z, w; };
struct uint2 { unsigned x, y; };
struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
static inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
static inline int2 make_int2(int a, int b) { return int2{a, b}; }
static inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
static inline uint2 make_uint2(unsigned a, unsigned b) { return uint2{a, b}; }
static inline float2 make_float2(float a, float b) { return float2{a, b}; }

namespace simt {
struct Fiber;
extern Fiber* cur;
extern uint3s g_block, g_bdim, g_gdim;
uint3s& tidx();
int lane_id();
enum Op { OP_BALLOT, OP_SHFL, OP_SHFL_UP, OP_SHFL_DOWN, OP_SHFL_XOR, OP_WBAR };
long long wave_op(int op, long long v, int arg);
void sync_block();
void yield();
void run_launch(dim3 g, dim3 b, void (*tramp)(void*), void* ctx, bool coop);
template <class F>
void launch(dim3 g, dim3 b, F f, bool coop = false) {
    run_launch(g, b, [](void* c) { (*(F*)c)(); }, (void*)&f, coop);
}
}  // namespace simt

#define threadIdx (::simt::tidx())
#define blockIdx (::simt::g_block)
#define blockDim (::simt::g_bdim)
#define gridDim (::simt::g_gdim)

static inline void __syncthreads() { ::simt::sync_block(); }
static inline unsigned __lane_id() { return (unsigned)::simt::lane_id(); }
static inline unsigned long long __ballot(int p) { return (unsigned long long)::simt::wave_op(::simt::OP_BALLOT, p != 0, 0); }
static inline int __any(int p) { return __ballot(p) != 0ull; }
static inline int __all(int p) {
    // every live lane
    return ::simt::wave_op(::simt::OP_BALLOT, p == 0, 0) == 0;
}
template <class T>
static inline long long simt_bits(T v) {
    long long b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
static inline T simt_unbits(long long b) {
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}
template <class T>
static inline T __shfl(T v, int src, int width = 64) {
    (void)width;
    return simt_unbits<T>(::simt::wave_op(::simt::OP_SHFL, simt_bits(v), src));
}
template <class T>
static inline T __shfl_up(T v, unsigned d, int width = 64) {
    (void)width;
    return simt_unbits<T>(::simt::wave_op(::simt::OP_SHFL_UP, simt_bits(v), (int)d));
}
template <class T>
static inline T __shfl_down(T v, unsigned d, int width = 64) {
    (void)width;
    return simt_unbits<T>(::simt::wave_op(::simt::OP_SHFL_DOWN, simt_bits(v), (int)d));
}
template <class T>
static inline T __shfl_xor(T v, int d, int width = 64) {
    (void)width;
    return simt_unbits<T>(::simt::wave_op(::simt::OP_SHFL_XOR, simt_bits(v), d));
}
#define __popcll(x) __builtin_popcountll((unsigned long long)(x))
#define __popc(x) __builtin_popcount((unsigned)(x))
#define __ffsll(x) __builtin_ffsll((long long)(x))
#define __ffs(x) __builtin_ffs((int)(x))
#define __clzll(x) ((x) ? __builtin_clzll((unsigned long long)(x)) : 64)
#define __clz(x) ((x) ? __builtin_clz((unsigned)(x)) : 32)

static inline unsigned simt_mbcnt_lo(unsigned m, unsigned acc) {
    int l = ::simt::lane_id();
    unsigned mask = l >= 32 ? 0xffffffffu : ((1u << l) - 1u);
    return acc + __builtin_popcount(m & mask);
}
static inline unsigned simt_mbcnt_hi(unsigned m, unsigned acc) {
    int l = ::simt::lane_id();
    unsigned mask = l < 32 ? 0u : (l == 63 ? 0x7fffffffu : ((1u << (l - 32)) - 1u));
    if (l >= 32 && l < 63) mask = (1u << (l - 32)) - 1u;
    return acc + __builtin_popcount(m & mask);
}
// DPP row shifts and row broadcasts (the controls the sweep uses): the value
// of the source lane, or old where the source lies outside the lane's row or
// the lane's row or bank is masked off.  Every lane of the wave takes part.
// (One call site for the shuffle and a select after it: a branch after the
// call lets the compiler copy the call into each path, which the divergence
// check would see as different sites.)
__attribute__((noinline)) static int simt_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                                                     bool bound_ctrl) {
    const int l = ::simt::lane_id(), row = l >> 4, bank = (l & 15) >> 2;
    int from = -1;
    if (ctrl > 0x110 && ctrl < 0x120) {
        const int d = ctrl - 0x110;
        if ((l & 15) >= d) from = l - d;
    } else if (ctrl == 0x142) {
        if (row >= 1) from = row * 16 - 1;
    } else if (ctrl == 0x143) {
        if (row >= 2) from = 31;
    } else {
        __builtin_trap();
    }
    const int v = __shfl(src, from < 0 ? l : from);
    const bool on = ((row_mask >> row) & 1) && ((bank_mask >> bank) & 1);
    const int off = bound_ctrl ? 0 : old;
    return on ? (from < 0 ? off : v) : old;
}
#define __builtin_amdgcn_update_dpp(o, s, c, rm, bm, bc) simt_update_dpp((o), (s), (c), (rm), (bm), (bc))
#define __builtin_amdgcn_mbcnt_lo(m, a) simt_mbcnt_lo((m), (a))
#define __builtin_amdgcn_mbcnt_hi(m, a) simt_mbcnt_hi((m), (a))
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() ((void)::simt::wave_op(::simt::OP_WBAR, 0, 0))
#define __builtin_amdgcn_s_sleep(x) (::simt::yield())
#define __builtin_amdgcn_s_waitcnt(x) ((void)(x))
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))

#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4

template <class T, class U>
static inline bool __hip_atomic_compare_exchange_strong(T* p, T* expected, U desired, int, int, int) {
    if (*p == *expected) {
        *p = (T)desired;
        return true;
    }
    *expected = *p;
    return false;
}
template <class T, class U>
static inline T __hip_atomic_fetch_max(T* p, U v, int, int) {
    T o = *p;
    if ((T)v > o) *p = (T)v;
    return o;
}
template <class T, class U>
static inline T __hip_atomic_fetch_min(T* p, U v, int, int) {
    T o = *p;
    if ((T)v < o) *p = (T)v;
    return o;
}
template <class T, class U>
static inline T __hip_atomic_fetch_add(T* p, U v, int, int) {
    T o = *p;
    *p = (T)(o + (T)v);
    return o;
}
template <class T, class U>
static inline T __hip_atomic_fetch_or(T* p, U v, int, int) {
    T o = *p;
    *p = (T)(o | (T)v);
    return o;
}
template <class T, class U>
static inline T __hip_atomic_fetch_and(T* p, U v, int, int) {
    T o = *p;
    *p = (T)(o & (T)v);
    return o;
}
template <class T, class U>
static inline T __hip_atomic_exchange(T* p, U v, int, int) {
    T o = *p;
    *p = (T)v;
    return o;
}
template <class T>
static inline T __hip_atomic_load(T* p, int, int) { return *p; }
template <class T, class U>
static inline void __hip_atomic_store(T* p, U v, int, int) { *p = (T)v; }

template <class T, class U>
static inline T atomicMax(T* p, U v) { return __hip_atomic_fetch_max(p, v, 0, 0); }
template <class T, class U>
static inline T atomicMin(T* p, U v) { return __hip_atomic_fetch_min(p, v, 0, 0); }
template <class T, class U>
static inline T atomicAdd(T* p, U v) { return __hip_atomic_fetch_add(p, v, 0, 0); }
template <class T, class U>
static inline T atomicSub(T* p, U v) { T o = *p; *p = (T)(o - (T)v); return o; }
template <class T, class U>
static inline T atomicOr(T* p, U v) { return __hip_atomic_fetch_or(p, v, 0, 0); }
template <class T, class U>
static inline T atomicAnd(T* p, U v) { return __hip_atomic_fetch_and(p, v, 0, 0); }
template <class T, class U>
static inline T atomicExch(T* p, U v) { return __hip_atomic_exchange(p, v, 0, 0); }
template <class T, class U, class V>
static inline T atomicCAS(T* p, U cmp, V val) {
    T o = *p;
    if (o == (T)cmp) *p = (T)val;
    return o;
}


static inline int min(int a, int b) { return a < b ? a : b; }
static inline int max(int a, int b) { return a > b ? a : b; }
static inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
static inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
static inline long long min(long long a, long long b) { return a < b ? a : b; }
static inline long long max(long long a, long long b) { return a > b ? a : b; }
static inline unsigned long long min(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
static inline unsigned long long max(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
static inline long min(long a, long b) { return a < b ? a : b; }
static inline long max(long a, long b) { return a > b ? a : b; }
static inline float min(float a, float b) { return a < b ? a : b; }
static inline float max(float a, float b) { return a > b ? a : b; }

#define __log2f(x) log2f(x)
#define __expf(x) expf(x)
#define __logf(x) logf(x)
static inline float __uint_as_float(unsigned u) { float f; memcpy(&f, &u, 4); return f; }
static inline unsigned __float_as_uint(float f) { unsigned u; memcpy(&u, &f, 4); return u; }
static inline int __float_as_int(float f) { int u; memcpy(&u, &f, 4); return u; }
static inline float __int_as_float(int u) { float f; memcpy(&f, &u, 4); return f; }
static inline long long clock64() { return 0; }
static inline long long wall_clock64() { return 0; }
static inline void __threadfence() {}
static inline void __threadfence_block() {}

// ---------------------------------------------------------------- host runtime
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;
typedef int hipMemcpyKind;
enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3,
       hipMemcpyDefault = 4 };
struct hipDeviceProp_t {
    int multiProcessorCount;
    int maxThreadsPerBlock;
    size_t sharedMemPerBlock;
    char gcnArchName[256];
    char name[256];
};
hipError_t simt_malloc(void** p, size_t bytes);
static inline hipError_t hipMalloc(void** p, size_t b) { return simt_malloc(p, b); }
template <class T>
static inline hipError_t hipMalloc(T** p, size_t b) { return simt_malloc((void**)p, b); }
hipError_t hipFree(void* p);
static inline hipError_t hipHostMalloc(void** p, size_t b, unsigned = 0) { *p = malloc(b); return *p ? 0 : 2; }
template <class T>
static inline hipError_t hipHostMalloc(T** p, size_t b, unsigned f = 0) { return hipHostMalloc((void**)p, b, f); }
static inline hipError_t hipHostFree(void* p) { free(p); return 0; }
static inline hipError_t hipMemcpy(void* d, const void* s, size_t b, hipMemcpyKind) { memmove(d, s, b); return 0; }
static inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t b, hipMemcpyKind, hipStream_t = 0) { memmove(d, s, b); return 0; }
static inline hipError_t hipMemsetAsync(void* d, int v, size_t b, hipStream_t = 0) { memset(d, v, b); return 0; }
static inline hipError_t hipMemset(void* d, int v, size_t b) { memset(d, v, b); return 0; }
static inline hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
static inline hipError_t hipDeviceSynchronize() { return 0; }
static inline hipError_t hipGetLastError() { return 0; }
static inline hipError_t hipPeekAtLastError() { return 0; }
static inline const char* hipGetErrorString(hipError_t) { return "simt"; }
static inline hipError_t hipGetDevice(int* d) { *d = 0; return 0; }
static inline hipError_t hipSetDevice(int) { return 0; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int dev);
static inline hipError_t hipEventCreate(hipEvent_t* e) { static char dummy[1024]; static int k; *e = &dummy[(k++) & 1023]; return 0; }
static inline hipError_t hipEventDestroy(hipEvent_t) { return 0; }
static inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = 0) { return 0; }
static inline hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
static inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.001f; return 0; }
enum { hipDeviceAttributeCooperativeLaunch = 1 };
static inline hipError_t hipDeviceGetAttribute(int* v, int attr, int) {
    *v = attr == hipDeviceAttributeCooperativeLaunch ? 1 : 0;
    return 0;
}
// Cooperative launch: every workgroup of the grid is live at once (the
// emulation interleaves them), and each calls the kernel with the arguments
// the pointers in args refer to.
template <class... A, size_t... I>
static inline void simt_coop_impl(void (*k)(A...), dim3 g, dim3 b, void** args, std::index_sequence<I...>) {
    ::simt::launch(g, b, [=]() { k(*static_cast<std::decay_t<A>*>(args[I])...); }, true);
}
template <class... A>
static inline hipError_t simt_coop(void (*k)(A...), dim3 g, dim3 b, void** args) {
    simt_coop_impl(k, g, b, args, std::index_sequence_for<A...>{});
    return 0;
}
#define hipLaunchCooperativeKernel(k, g, b, args, sm, st) simt_coop(k, dim3(g), dim3(b), (args))

#define hipLaunchKernelGGL(k, g, b, sm, st, ...) ::simt::launch(dim3(g), dim3(b), [=]() { k(__VA_ARGS__); })
