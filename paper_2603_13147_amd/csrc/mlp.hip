// mlp.hip - the learned scheduler's network on gfx950: forward, loss,
// backward and Adam kernels for training, and the per-round trace features.
//
// Network: 12 round features -> 64 -> 64 -> 5 outputs, ReLU hidden layers.
// Weights are kept in FP32 (master copy) and used as BF16 (round to nearest
// even) in every product; inputs and hidden activations are rounded to BF16;
// accumulation is FP32.  The outputs are a push logit, a dense logit and
// three delta-class logits.  One wave evaluates one row, lane j owning hidden
// unit j in both layers; the backward pass keeps each lane's gradient rows in
// registers across the rows of its wave, reduces the waves of a workgroup in
// LDS and adds one value per parameter and workgroup to the global gradient.
//
// The features of a traced round are computed by the same device function the
// sweep uses when it decides that round, so a network trained on trace
// features sees exactly the inputs it is given at decision time.
#include <math.h>
#include <string.h>

#include "llp_host.h"
#include "llp_sched.h"

namespace llp {

constexpr int NI = LLP_MLP_IN, NH = LLP_MLP_HID, NO = LLP_MLP_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NO * NH, NPAR = OFF_B3 + NO;
static_assert(NPAR == LLP_MLP_PARAMS, "parameter layout");

__device__ __forceinline__ float bfw(const float* p, int i) { return round_bf16(p[i]); }

constexpr int MB = 256;            // threads per workgroup
constexpr int MW = MB / LLP_WAVE;  // waves per workgroup

// act[row][0..63] = h1, act[row][64..127] = h2 (bf16 bits)
__global__ void __launch_bounds__(MB) k_mlp_forward(int B, const float* P, const float* X, float* logits,
                                                    unsigned short* act) {
    const int j = lane();
    const int wave = blockIdx.x * MW + (threadIdx.x >> 6);
    const int nw = gridDim.x * MW;
    // this lane's weights as bf16-valued floats
    float w1[NI], w2[NH], w3[NO];
#pragma unroll
    for (int k = 0; k < NI; ++k) w1[k] = bfw(P, OFF_W1 + j * NI + k);
#pragma unroll
    for (int k = 0; k < NH; ++k) w2[k] = bfw(P, OFF_W2 + j * NH + k);
#pragma unroll
    for (int o = 0; o < NO; ++o) w3[o] = bfw(P, OFF_W3 + o * NH + j);
    const float b1 = bfw(P, OFF_B1 + j), b2 = bfw(P, OFF_B2 + j);
    for (int row = wave; row < B; row += nw) {
        const float* x = X + (long long)row * NI;
        float a = b1;
#pragma unroll
        for (int k = 0; k < NI; ++k) a += w1[k] * round_bf16(x[k]);
        const float h1 = round_bf16(fmaxf(a, 0.f));
        float a2 = b2;
#pragma unroll
        for (int k = 0; k < NH; ++k) a2 += w2[k] * __shfl(h1, k, LLP_WAVE);
        const float h2 = round_bf16(fmaxf(a2, 0.f));
        act[(long long)row * 2 * NH + j] = f32_to_bf16(h1);
        act[(long long)row * 2 * NH + NH + j] = f32_to_bf16(h2);
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            float t = w3[o] * h2;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, LLP_WAVE);
            if (j == 0) logits[(long long)row * NO + o] = t + bfw(P, OFF_B3 + o);
        }
    }
}

// Loss over the batch (one workgroup, deterministic): mean of
// BCE(o0, push) + BCE(o1, dense) + softmax-CE(o2..o4, delta class).
// labels are round codes: mode in bits 0-1 (2 = push, 1 = dense), delta class
// in bits 8-9.  dlogits = d loss / d logits.
__global__ void __launch_bounds__(1024) k_mlp_loss(int B, const float* L, const int* labels, float* dL,
                                                   float* loss) {
    __shared__ float part[1024 / LLP_WAVE];
    float acc = 0.f;
    const float inv = 1.f / (float)(B > 0 ? B : 1);
    for (int row = threadIdx.x; row < B; row += blockDim.x) {
        const float* o = L + (long long)row * NO;
        float* d = dL + (long long)row * NO;
        const int code = labels[row];
        const int mode = code & 3, dc = min((code >> 8) & 3, 2);
        const float y0 = mode == 2 ? 1.f : 0.f, y1 = mode == 1 ? 1.f : 0.f;
        // numerically stable BCE with logits: max(o,0) - o*y + log(1 + exp(-|o|))
        float l = 0.f;
        for (int k = 0; k < 2; ++k) {
            const float z = o[k], y = k == 0 ? y0 : y1;
            l += fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)));
            const float s = 1.f / (1.f + expf(-z));
            d[k] = (s - y) * inv;
        }
        const float mx = fmaxf(o[2], fmaxf(o[3], o[4]));
        const float e2 = expf(o[2] - mx), e3 = expf(o[3] - mx), e4 = expf(o[4] - mx);
        const float se = e2 + e3 + e4;
        const float lse = mx + logf(se);
        l += lse - o[2 + dc];
        d[2] = (e2 / se - (dc == 0 ? 1.f : 0.f)) * inv;
        d[3] = (e3 / se - (dc == 1 ? 1.f : 0.f)) * inv;
        d[4] = (e4 / se - (dc == 2 ? 1.f : 0.f)) * inv;
        acc += l;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, LLP_WAVE);
    if (lane() == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
        *loss = t * inv;
    }
}

// Backward: grad += d loss / d params (straight through the bf16 rounding).
__global__ void __launch_bounds__(MB) k_mlp_backward(int B, const float* P, const float* X,
                                                     const unsigned short* act, const float* dL, float* grad) {
    __shared__ float red[NPAR];
    const int j = lane();
    const int wv = threadIdx.x >> 6;
    const int wave = blockIdx.x * MW + wv;
    const int nw = gridDim.x * MW;
    for (int i = threadIdx.x; i < NPAR; i += MB) red[i] = 0.f;
    // lane j: column j of W2 (for dh1[j]) and column j of W3 (for dh2[j])
    float w2c[NH], w3c[NO];
#pragma unroll
    for (int k = 0; k < NH; ++k) w2c[k] = bfw(P, OFF_W2 + k * NH + j);
#pragma unroll
    for (int o = 0; o < NO; ++o) w3c[o] = bfw(P, OFF_W3 + o * NH + j);
    float gW1[NI], gW2[NH], gW3[NO], gb3[NO];
    float gb1 = 0.f, gb2 = 0.f;
#pragma unroll
    for (int k = 0; k < NI; ++k) gW1[k] = 0.f;
#pragma unroll
    for (int k = 0; k < NH; ++k) gW2[k] = 0.f;
#pragma unroll
    for (int o = 0; o < NO; ++o) gW3[o] = gb3[o] = 0.f;
    for (int row = wave; row < B; row += nw) {
        const float h1 = bf16_to_f32(act[(long long)row * 2 * NH + j]);
        const float h2 = bf16_to_f32(act[(long long)row * 2 * NH + NH + j]);
        float d[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) d[o] = dL[(long long)row * NO + o];
        // layer 3: logits = W3 h2 + b3
        float dh2 = 0.f;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            gW3[o] += d[o] * h2;
            gb3[o] += d[o];
            dh2 += w3c[o] * d[o];
        }
        const float dz2 = h2 > 0.f ? dh2 : 0.f;
        gb2 += dz2;
        // lane j holds row j of W2's gradient: dz2[j] * h1[k]
#pragma unroll
        for (int k = 0; k < NH; ++k) gW2[k] += dz2 * __shfl(h1, k, LLP_WAVE);
        // dh1[j] = sum_k W2[k][j] dz2[k]
        float dh1 = 0.f;
#pragma unroll
        for (int k = 0; k < NH; ++k) dh1 += w2c[k] * __shfl(dz2, k, LLP_WAVE);
        const float dz1 = h1 > 0.f ? dh1 : 0.f;
        gb1 += dz1;
        const float* x = X + (long long)row * NI;
#pragma unroll
        for (int k = 0; k < NI; ++k) gW1[k] += dz1 * round_bf16(x[k]);
    }
    __syncthreads();
    // reduce the workgroup's waves in LDS
#pragma unroll
    for (int k = 0; k < NI; ++k) atomicAdd(&red[OFF_W1 + j * NI + k], gW1[k]);
    atomicAdd(&red[OFF_B1 + j], gb1);
#pragma unroll
    for (int k = 0; k < NH; ++k) atomicAdd(&red[OFF_W2 + j * NH + k], gW2[k]);
    atomicAdd(&red[OFF_B2 + j], gb2);
#pragma unroll
    for (int o = 0; o < NO; ++o) atomicAdd(&red[OFF_W3 + o * NH + j], gW3[o]);
    if (j == 0) {
#pragma unroll
        for (int o = 0; o < NO; ++o) atomicAdd(&red[OFF_B3 + o], gb3[o]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NPAR; i += MB)
        if (red[i] != 0.f) atomicAdd(&grad[i], red[i]);
}

__global__ void k_mlp_adam(const float* g, float* p, float* m1, float* m2, int step, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// features[r][12] of traced rounds r = 1..rounds, as the sweep computes them
// when it decides round r (history from the record of round r-1; the
// hybrid's code for the round from the same parameters the sweep uses).
__global__ void k_trace_features(long long rounds, const llp_trace_rec* tr, int n, int m, SchedParams sp, float* F) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    SchedHist h;
    memset(&h, 0, sizeof(h));
    for (long long r = 1; r <= rounds; ++r) {
        const llp_trace_rec t = tr[r - 1];
        float f[12];
        round_features(f, (int)r, t.in_count, (int)t.in_edges, n, m, h, hybrid_code(sp, (int)t.in_edges, m));
        for (int k = 0; k < 12; ++k) F[(r - 1) * 12 + k] = f[k];
        const long long prev_adv = h.adv_total;
        h.r = (int)r;
        h.mode = t.mode & 3;
        h.cl_count = t.in_count;
        h.cl_edges = (int)t.in_edges;
        h.wl_count = t.out_count;
        h.wl_edges = (int)t.out_edges;
        h.adv_total = prev_adv + t.in_count;
    }
}

static int mlp_grid(int B) {
    int g = (B + MW - 1) / MW;
    int cap = device_info().cus * 4;
    if (g > cap) g = cap;
    return g < 1 ? 1 : g;
}

}  // namespace llp

extern "C" {

int llp_mlp_forward(int32_t B, const float* params, const float* x, float* logits, uint16_t* act, void* stream) {
    if (B < 0 || !params || (B > 0 && (!x || !logits || !act))) return llp::fail(LLP_E_ARG, "bad forward arguments");
    if (B == 0) return LLP_OK;
    hipLaunchKernelGGL(llp::k_mlp_forward, dim3(llp::mlp_grid(B)), dim3(llp::MB), 0, (hipStream_t)stream, B, params,
                       x, logits, act);
    return llp::hip_check(hipGetLastError(), "k_mlp_forward");
}

int llp_mlp_loss(int32_t B, const float* logits, const int32_t* labels, float* dlogits, float* loss, void* stream) {
    if (B < 0 || !loss || (B > 0 && (!logits || !labels || !dlogits))) return llp::fail(LLP_E_ARG, "bad loss arguments");
    hipLaunchKernelGGL(llp::k_mlp_loss, dim3(1), dim3(1024), 0, (hipStream_t)stream, B, logits, labels, dlogits, loss);
    return llp::hip_check(hipGetLastError(), "k_mlp_loss");
}

int llp_mlp_backward(int32_t B, const float* params, const float* x, const uint16_t* act, const float* dlogits,
                     float* grad, void* stream) {
    if (B < 0 || !params || !grad || (B > 0 && (!x || !act || !dlogits)))
        return llp::fail(LLP_E_ARG, "bad backward arguments");
    if (B == 0) return LLP_OK;
    hipLaunchKernelGGL(llp::k_mlp_backward, dim3(llp::mlp_grid(B)), dim3(llp::MB), 0, (hipStream_t)stream, B,
                       params, x, act, dlogits, grad);
    return llp::hip_check(hipGetLastError(), "k_mlp_backward");
}

int llp_mlp_adam(const float* grad, float* params, float* m1, float* m2, int32_t step, float lr, void* stream) {
    if (!grad || !params || !m1 || !m2 || step < 1) return llp::fail(LLP_E_ARG, "bad Adam arguments");
    hipLaunchKernelGGL(llp::k_mlp_adam, dim3((LLP_MLP_PARAMS + 255) / 256), dim3(256), 0, (hipStream_t)stream, grad,
                       params, m1, m2, step, lr);
    return llp::hip_check(hipGetLastError(), "k_mlp_adam");
}

int llp_trace_features(int64_t rounds, const llp_trace_rec* trace, int32_t n, int64_t m, int32_t kind,
                       float* features, void* stream) {
    if (rounds < 0 || n <= 0 || m < 0 || m > 0x7fffffffll || (rounds > 0 && (!trace || !features)))
        return llp::fail(LLP_E_ARG, "bad trace-feature arguments");
    if (kind != LLP_KIND_SSSP && kind != LLP_KIND_BFS && kind != LLP_KIND_JOBS)
        return llp::fail(LLP_E_ARG, "kind must be LLP_KIND_SSSP, LLP_KIND_BFS or LLP_KIND_JOBS");
    if (rounds == 0) return LLP_OK;
    llp::SchedParams sp;
    memset(&sp, 0, sizeof(sp));
    llp::hybrid_params(kind, n, m, true, &sp);
    hipLaunchKernelGGL(llp::k_trace_features, dim3(1), dim3(64), 0, (hipStream_t)stream, (long long)rounds, trace, n,
                       (int)m, sp, features);
    return llp::hip_check(hipGetLastError(), "k_trace_features");
}

}  // extern "C"
