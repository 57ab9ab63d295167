// llp_host.cpp - host-side plumbing of libllp (errors, device info,
// workspace, pinned readback) and the small library-wide entry points.
#include "llp_host.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>

namespace llp {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return LLP_OK;
    set_error("HIP error in %s: %s", what, hipGetErrorString(e));
    return LLP_E_HIP;
}

static std::mutex g_mu;
static std::map<int, DeviceInfo> g_dev;

const DeviceInfo& device_info() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) return it->second;
    hipDeviceProp_t p;
    memset(&p, 0, sizeof(p));
    (void)hipGetDeviceProperties(&p, dev);
    DeviceInfo d;
    d.device = dev;
    d.cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 1;
    d.max_threads = p.maxThreadsPerBlock;
    d.lds_per_block = p.sharedMemPerBlock;
    d.arch = p.gcnArchName;
    return g_dev.emplace(dev, d).first->second;
}

llp_opts opts_or_default(const llp_opts* o) {
    llp_opts d;
    memset(&d, 0, sizeof(d));
    d.size = sizeof(llp_opts);
    if (o) {
        size_t n = o->size ? (o->size < sizeof(llp_opts) ? o->size : sizeof(llp_opts)) : sizeof(llp_opts);
        memcpy(&d, o, n);
    }
    return d;
}

struct OwnedWs {
    void* ptr = nullptr;
    size_t bytes = 0;
};
static std::map<int, OwnedWs> g_ws;

int get_workspace(const llp_opts& o, size_t bytes, void** out) {
    if (o.workspace) {
        if (o.workspace_bytes < bytes)
            return fail(LLP_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes needed",
                        o.workspace_bytes, bytes);
        *out = o.workspace;
        return LLP_OK;
    }
    int dev = 0;
    LLP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    OwnedWs& w = g_ws[dev];
    if (w.bytes < bytes) {
        if (w.ptr) {
            LLP_HIP(hipDeviceSynchronize());
            LLP_HIP(hipFree(w.ptr));
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        LLP_HIP(hipMalloc(&w.ptr, want));
        w.bytes = want;
    }
    *out = w.ptr;
    return LLP_OK;
}

struct Pinned {
    void* ptr = nullptr;
    size_t bytes = 0;
};
static thread_local std::map<int, Pinned> t_pinned;

void* pinned_scratch(size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    Pinned& p = t_pinned[dev];
    if (p.bytes < bytes) {
        if (p.ptr) (void)hipHostFree(p.ptr);
        p.ptr = nullptr;
        p.bytes = 0;
        size_t want = bytes < 4096 ? 4096 : bytes;
        if (hipHostMalloc(&p.ptr, want, 0) != hipSuccess) return nullptr;
        p.bytes = want;
    }
    return p.ptr;
}

int readback(hipStream_t s, const void* src, void* dst, size_t bytes) {
    void* pin = pinned_scratch(bytes);
    if (!pin) return fail(LLP_E_HIP, "pinned host allocation failed");
    LLP_HIP(hipMemcpyAsync(pin, src, bytes, hipMemcpyDeviceToHost, s));
    LLP_HIP(hipStreamSynchronize(s));
    memcpy(dst, pin, bytes);
    return LLP_OK;
}

void batch_release();

}  // namespace llp

extern "C" {

const char* llp_last_error(void) { return llp::g_err; }

const char* llp_version(void) { return "libllp 0.1 (gfx950)"; }

void llp_shutdown(void) {
    llp::batch_release();
    std::lock_guard<std::mutex> lk(llp::g_mu);
    for (auto& kv : llp::g_ws) {
        if (kv.second.ptr) {
            (void)hipSetDevice(kv.first);
            (void)hipDeviceSynchronize();
            (void)hipFree(kv.second.ptr);
        }
    }
    llp::g_ws.clear();
}

}  // extern "C"
