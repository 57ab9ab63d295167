// sched_host.cpp - host side of the per-round schedulers: option checking
// and the device copy of the learned scheduler's weights.
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "llp_host.h"
#include "llp_sched.h"

namespace llp {

static std::mutex g_wmu;
static std::map<int, unsigned short*> g_w;   // device -> bf16 parameter block

static unsigned short host_bf16(float f) {
    unsigned u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (unsigned short)(u >> 16);
}

const unsigned short* learned_weights_device() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_wmu);
    auto it = g_w.find(dev);
    return it == g_w.end() ? nullptr : it->second;
}

int sched_params(const llp_opts& o, bool can_push, SchedParams* sp) {
    memset(sp, 0, sizeof(*sp));
    sp->sched = o.sched;
    sp->flags = o.flags;
    sp->delta = o.delta;
    sp->can_push = can_push ? 1 : 0;
    sp->seed = o.seed;
    sp->dense_frac = 0.5f;
    sp->push_dclass = DCLS_NONE;
    if (o.sched == LLP_SCHED_SCRIPT) {
        if (o.plan_len < 0 || (o.plan_len > 0 && !o.plan)) return fail(LLP_E_ARG, "SCRIPT needs plan and plan_len");
        sp->plan = o.plan;
        sp->plan_len = o.plan_len;
    }
    if (o.delta < 0) return fail(LLP_E_ARG, "delta must be >= 0");
    if (o.sched == LLP_SCHED_LEARNED) {
        sp->mlp = learned_weights_device();
        if (!sp->mlp) return fail(LLP_E_ARG, "LLP_SCHED_LEARNED needs llp_sched_set_weights() first");
    }
    return LLP_OK;
}

void hybrid_params(int kind, long long n, long long m, bool can_push, SchedParams* sp) {
    // BFS dense rounds skip the rows already final (the level cap), so they pay
    // from a much narrower frontier: m / 14 (the direction-optimizing BFS
    // threshold); weighted dense rounds gather only the arcs that pass the arc
    // bound and switch at m / 3 (on R-MAT 22 a dense round costs what a push of
    // about 0.37 m arcs does); jobs at m / 2
    sp->dense_frac = kind == LLP_KIND_BFS ? 1.0f / 14.0f : (kind == LLP_KIND_SSSP ? 1.0f / 3.0f : 0.5f);
    sp->can_push = can_push ? 1 : 0;
    // sparse weighted graphs with several arcs per vertex (a mesh): unbucketed
    // push rounds re-correct each distance many times (about 200 advances per
    // vertex on the 4096^2 grid), wide buckets settle it in about five; below
    // two arcs per vertex (chains) there is little to re-correct and buckets
    // only add rounds
    sp->push_dclass =
        (kind == LLP_KIND_SSSP && can_push && n > 0 && m >= 2 * n && m < 8 * n) ? DCLS_WIDE : DCLS_NONE;
}

}  // namespace llp

extern "C" int llp_sched_set_weights(const float* params) {
    if (!params) return llp::fail(LLP_E_ARG, "params is NULL");
    std::vector<unsigned short> h(LLP_MLP_PARAMS);
    for (int i = 0; i < LLP_MLP_PARAMS; ++i) h[i] = llp::host_bf16(params[i]);
    int dev = 0;
    LLP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(llp::g_wmu);
    unsigned short*& d = llp::g_w[dev];
    if (!d) LLP_HIP(hipMalloc(&d, sizeof(unsigned short) * LLP_MLP_PARAMS));
    LLP_HIP(hipMemcpy(d, h.data(), sizeof(unsigned short) * LLP_MLP_PARAMS, hipMemcpyHostToDevice));
    return LLP_OK;
}
