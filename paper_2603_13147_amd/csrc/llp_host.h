// llp_host.h - host-side plumbing shared by the C ABI entry points: error
// reporting, option defaults, per-device properties, workspace carving and
// the pinned readback buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/llp.h"

namespace llp {

// thread-local message for llp_last_error()
void set_error(const char* fmt, ...);
int fail(int status, const char* fmt, ...);

// returns LLP_E_HIP with a message if e != hipSuccess
int hip_check(hipError_t e, const char* what);
#define LLP_HIP(call)                                          \
    do {                                                       \
        int _s = ::llp::hip_check((call), #call);              \
        if (_s) return _s;                                     \
    } while (0)

struct DeviceInfo {
    int device;
    int cus;
    int max_threads;
    size_t lds_per_block;
    std::string arch;
};
const DeviceInfo& device_info();

// Autotuner records (tune.cpp), per (architecture, CU count, kind, size
// class = floor(log2(size))) of the current device.
int size_class(long long size);
void tune_record(int kind, long long size, int block, int chunk);
bool tune_lookup(int kind, long long size, int* block, int* chunk);   // own class, else the nearest
bool tune_last(int kind, int* block, int* chunk);                      // the most recent record
void tune_clear();

// copy of opts with defaults filled in
llp_opts opts_or_default(const llp_opts* o);

// Workspace carving: a bump allocator over a caller-provided or
// library-owned device buffer (256-byte aligned pieces).
struct Carver {
    char* base;
    size_t cap;
    size_t used = 0;
    bool measure_only;
    template <class T>
    T* take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        size_t at = used;
        used += bytes;
        if (measure_only || used > cap) return nullptr;
        return reinterpret_cast<T*>(base + at);
    }
};

// Resolve the workspace for a solve needing `bytes`: the caller's buffer
// (LLP_E_WORKSPACE if too small) or a library-owned one (grown on demand,
// per device).  *out receives the device pointer.
int get_workspace(const llp_opts& o, size_t bytes, void** out);

// Small pinned host buffer per thread and device, for status readback.
void* pinned_scratch(size_t bytes);

// Wait for the stream and read `bytes` from device pointer src into dst via the
// pinned scratch buffer.
int readback(hipStream_t s, const void* src, void* dst, size_t bytes);

}  // namespace llp
