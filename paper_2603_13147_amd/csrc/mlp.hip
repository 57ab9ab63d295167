// mlp.hip - the learned scheduler's network on gfx950: forward, loss,
// backward and Adam kernels for training, and the per-round trace features.
//
// Network: 12 round features -> 64 -> 64 -> 5 outputs, ReLU hidden layers.
// Weights are kept in FP32 (master copy) and used as BF16 (round to nearest
// even) in every product; inputs and hidden activations are rounded to BF16;
// accumulation is FP32.  The outputs are a push logit, a dense logit and
// three delta-class logits.
//
// Both training passes run on the matrix cores, one wave per tile of 16
// rows.  The forward pass is three BF16 products with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16): the BF16 inputs and weights are exactly the
// values the network defines, and the products of two BF16 values are exact
// in FP32.  Each hidden layer goes through the wave's LDS tile between the
// accumulator layout of one product and the operand layout of the next.
// The backward pass keeps the gradient signals in FP32 (the straight-through
// rule passes them unrounded), so its products are FP32 ones
// (v_mfma_f32_16x16x4_f32): dH2 = dL W3, dH1 = dZ2 W2, and the weight
// gradients dZ^T H summed over the wave's tiles in accumulators; the waves
// of a workgroup are reduced in LDS and each workgroup adds one value per
// parameter to the global gradient.
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
constexpr int MT = 16;             // rows per tile (the matrix products' M)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operand layouts of the two products, for lane l (wave64):
//   16x16x16 bf16: A[i][k] at i = l % 16, k = 4 (l / 16) + q (q = 0..3);
//                  B[k][j] at k = 4 (l / 16) + q, j = l % 16
//   16x16x4 f32:   A[i][k] at i = l % 16, k = l / 16; B[k][j] at k = l / 16, j = l % 16
//   both:          D[i][j] at i = 4 (l / 16) + q, j = l % 16
__device__ __forceinline__ f32x4 mma_bf16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ short bfbits(float f) { return (short)f32_to_bf16(f); }

// act[row][0..63] = h1, act[row][64..127] = h2 (bf16 bits)
__global__ void __launch_bounds__(MB) k_mlp_forward(int B, const float* P, const float* X, float* logits,
                                                    unsigned short* act) {
    __shared__ unsigned short hs[MW][MT * NH];   // one wave's hidden tile, row-major
    const int l = lane(), w = threadIdx.x >> 6;
    const int lr = l & 15, lg = l >> 4;          // operand row / column, and k group
    unsigned short* h = hs[w];
    // B operands (the transposed weights), as bf16
    bf16x4 bw1[4], bw2[4][4], bw3[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * lg + q, j = nt * 16 + lr;
            bw1[nt][q] = k < NI ? bfbits(P[OFF_W1 + j * NI + k]) : (short)0;
        }
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = ks * 16 + 4 * lg + q;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bw2[ks][nt][q] = bfbits(P[OFF_W2 + (nt * 16 + lr) * NH + k]);
            bw3[ks][q] = lr < NO ? bfbits(P[OFF_W3 + lr * NH + k]) : (short)0;
        }
    float b1[4], b2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        b1[nt] = bfw(P, OFF_B1 + nt * 16 + lr);
        b2[nt] = bfw(P, OFF_B2 + nt * 16 + lr);
    }
    const float b3 = lr < NO ? bfw(P, OFF_B3 + lr) : 0.f;
    const int ntiles = (B + MT - 1) / MT;
    for (int tile = blockIdx.x * MW + w; tile < ntiles; tile += gridDim.x * MW) {
        const long long r0 = (long long)tile * MT;
        // layer 1: X (16 x 12, padded to 16) times W1^T
        bf16x4 ax;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * lg + q;
            ax[q] = (r0 + lr < B && k < NI) ? bfbits(X[(r0 + lr) * NI + k]) : (short)0;
        }
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 d = mma_bf16(ax, bw1[nt], z);
#pragma unroll
            for (int q = 0; q < 4; ++q) h[(4 * lg + q) * NH + nt * 16 + lr] = f32_to_bf16(fmaxf(d[q] + b1[nt], 0.f));
        }
        // the hidden layers: the tile in LDS turns the accumulator layout into
        // the operand layout of the next product
        for (int layer = 0; layer < 2; ++layer) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            bf16x4 ah[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const unsigned short* src = h + lr * NH + ks * 16 + 4 * lg;
#pragma unroll
                for (int q = 0; q < 4; ++q) ah[ks][q] = (short)src[q];
            }
            // this layer's activations to act (rows of the tile inside the batch)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long long row = r0 + 4 * lg + q;
                if (row < B)
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        act[row * 2 * NH + layer * NH + nt * 16 + lr] = h[(4 * lg + q) * NH + nt * 16 + lr];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (layer == 0) {
                // layer 2: H1 W2^T
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    f32x4 d = z;
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) d = mma_bf16(ah[ks], bw2[ks][nt], d);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        h[(4 * lg + q) * NH + nt * 16 + lr] = f32_to_bf16(fmaxf(d[q] + b2[nt], 0.f));
                }
            } else {
                // layer 3: H2 W3^T (5 of 16 columns used)
                f32x4 d = z;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) d = mma_bf16(ah[ks], bw3[ks], d);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long long row = r0 + 4 * lg + q;
                    if (row < B && lr < NO) logits[row * NO + lr] = d[q] + b3;
                }
            }
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
// Per tile of 16 rows, with each wave's tiles in LDS as FP32 (rows past the
// batch are zero and contribute nothing):
//   dH2 = dL W3 (K = 5, padded to 8), dZ2 = dH2 where H2 > 0;
//   gW3 += dL^T H2, gW2 += dZ2^T H1;
//   dH1 = dZ2 W2 (W2 from LDS), dZ1 = dH1 where H1 > 0; gW1 += dZ1^T X;
//   the biases' gradients are the column sums of dL, dZ2 and dZ1.
struct BwdWave {
    float x[MT][16];              // bf16 inputs, columns 12..15 zero
    float d[MT][8];               // dL, columns 5..7 zero
    unsigned short h1[MT][NH];    // bf16 bits as stored by the forward pass
    unsigned short h2[MT][NH];
    float z[MT][NH];              // dZ2, then dZ1
};
struct BwdShared {
    float w2[NH * NH];  // bf16 W2, row-major [out][in]
    union {
        BwdWave wv[MW];
        float red[NPAR];
    };
};

static_assert(sizeof(BwdShared) <= 64 * 1024, "backward LDS within the default per-workgroup limit");

__global__ void __launch_bounds__(MB) k_mlp_backward(int B, const float* P, const float* X,
                                                     const unsigned short* act, const float* dL, float* grad) {
    extern __shared__ __align__(16) unsigned char smem[];
    BwdShared& sh = *reinterpret_cast<BwdShared*>(smem);
    const int l = lane(), w = threadIdx.x >> 6;
    const int lr = l & 15, lg = l >> 4;
    for (int i = threadIdx.x; i < NH * NH; i += MB) sh.w2[i] = bfw(P, OFF_W2 + i);
    // W3 as the B operand of dH2 = dL W3: B[k][j] = W3[k][j], k = ks * 4 + lg (< 5)
    float bw3[2][4];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int k = ks * 4 + lg;
            bw3[ks][nt] = k < NO ? bfw(P, OFF_W3 + k * NH + nt * 16 + lr) : 0.f;
        }
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 g2[4][4], g1[4], g3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        g1[a] = z;
        g3[a] = z;
#pragma unroll
        for (int b = 0; b < 4; ++b) g2[a][b] = z;
    }
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;   // lane l: column l (gb3: l < 5)
    __syncthreads();
    BwdWave& t = sh.wv[w];
    const int ntiles = (B + MT - 1) / MT;
    for (int tile = blockIdx.x * MW + w; tile < ntiles; tile += gridDim.x * MW) {
        const long long r0 = (long long)tile * MT;
        // the tile's rows into LDS: 64 lanes over 16 rows
        for (int i = l; i < MT * NH; i += LLP_WAVE) {
            const int row = i / NH, c = i % NH;
            const bool in = r0 + row < B;
            t.h1[row][c] = in ? act[(r0 + row) * 2 * NH + c] : (unsigned short)0;
            t.h2[row][c] = in ? act[(r0 + row) * 2 * NH + NH + c] : (unsigned short)0;
        }
        for (int i = l; i < MT * 16; i += LLP_WAVE) {
            const int row = i / 16, c = i % 16;
            t.x[row][c] = (r0 + row < B && c < NI) ? round_bf16(X[(r0 + row) * NI + c]) : 0.f;
        }
        for (int i = l; i < MT * 8; i += LLP_WAVE) {
            const int row = i / 8, c = i % 8;
            t.d[row][c] = (r0 + row < B && c < NO) ? dL[(r0 + row) * NO + c] : 0.f;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // dZ2 = (dL W3) where H2 > 0
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 d = z;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) d = mma_f32(t.d[lr][ks * 4 + lg], bw3[ks][nt], d);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * lg + q, c = nt * 16 + lr;
                t.z[row][c] = bf16_to_f32(t.h2[row][c]) > 0.f ? d[q] : 0.f;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW3 += dL^T H2 (rows of the output: 5 of 16) and gW2 += dZ2^T H1, K = the tile's rows
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = ks * 4 + lg;
            const float a3 = lr < 8 ? t.d[k][lr] : 0.f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                g3[nt] = mma_f32(a3, bf16_to_f32(t.h2[k][nt * 16 + lr]), g3[nt]);
                const float b = bf16_to_f32(t.h1[k][nt * 16 + lr]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) g2[mt][nt] = mma_f32(t.z[k][mt * 16 + lr], b, g2[mt][nt]);
            }
        }
        // bias gradients: column sums
        {
            float s2 = 0.f;
            for (int row = 0; row < MT; ++row) s2 += t.z[row][l];
            gb2 += s2;
        }
        if (l < NO) {
            float s3 = 0.f;
            for (int row = 0; row < MT; ++row) s3 += t.d[row][l];
            gb3 += s3;
        }
        // dZ1 = (dZ2 W2) where H1 > 0, into the dZ2 tile once every lane has read it
        f32x4 dh[4] = {z, z, z, z};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const float a = t.z[lr][ks * 4 + lg];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) dh[nt] = mma_f32(a, sh.w2[(ks * 4 + lg) * NH + nt * 16 + lr], dh[nt]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * lg + q, c = nt * 16 + lr;
                t.z[row][c] = bf16_to_f32(t.h1[row][c]) > 0.f ? dh[nt][q] : 0.f;
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // gW1 += dZ1^T X
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = ks * 4 + lg;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) g1[mt] = mma_f32(t.z[k][mt * 16 + lr], t.x[k][lr], g1[mt]);
        }
        {
            float s1 = 0.f;
            for (int row = 0; row < MT; ++row) s1 += t.z[row][l];
            gb1 += s1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // reduce the workgroup's waves in LDS (the tiles' space becomes the sums)
    __syncthreads();
    for (int i = threadIdx.x; i < NPAR; i += MB) sh.red[i] = 0.f;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 4 * lg + q;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) atomicAdd(&sh.red[OFF_W2 + (mt * 16 + r) * NH + nt * 16 + lr], g2[mt][nt][q]);
            if (r < NO) atomicAdd(&sh.red[OFF_W3 + r * NH + nt * 16 + lr], g3[nt][q]);
        }
        if (lr < NI)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) atomicAdd(&sh.red[OFF_W1 + (mt * 16 + r) * NI + lr], g1[mt][q]);
    }
    atomicAdd(&sh.red[OFF_B1 + l], gb1);
    atomicAdd(&sh.red[OFF_B2 + l], gb2);
    if (l < NO) atomicAdd(&sh.red[OFF_B3 + l], gb3);
    __syncthreads();
    for (int i = threadIdx.x; i < NPAR; i += MB)
        if (sh.red[i] != 0.f) atomicAdd(&grad[i], sh.red[i]);
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

// one wave per tile of MT rows
static int mlp_grid(int B) {
    int g = (B + MT * MW - 1) / (MT * MW);
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
    hipLaunchKernelGGL(llp::k_mlp_backward, dim3(llp::mlp_grid(B)), dim3(llp::MB), sizeof(llp::BwdShared),
                       (hipStream_t)stream, B, params, x, act, dlogits, grad);
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
