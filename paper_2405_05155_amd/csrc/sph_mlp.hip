// sph_mlp.hip -- the learned warm start of the relaxation: neighbour-offset
// features, a 100-128-128-3 GELU network on BF16 MFMA tiles with FP32
// accumulation, its training step (backward + AdamW on FP32 masters), and
// its application to a relaxing configuration.
//
// Rounding points (shared with the oracle): weights, layer inputs and the
// backward GEMM operands are rounded to BF16 (nearest-even); bias, GELU,
// loss and optimizer arithmetic are FP32.
//
// Two kernels carry the network: a forward pass and a fused training pass
// (forward, loss, backward and per-workgroup weight-gradient partials in one
// launch), both on v_mfma_f32_16x16x16_bf16 with the weights held in LDS,
// then a reduction of the partials in a fixed order (deterministic results)
// fused with the AdamW update.
#include "sph_internal.h"

#include <mutex>

namespace {

constexpr int NIN = 100, NH = 128, NOUT = 3;
constexpr int FS = SPH_MLP_FEAT_STRIDE;  // feature row stride (zero padded)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == SPH_MLP_NPARAMS, "parameter count");
constexpr int CHUNK = 1 << 18;  // feature rows per chunk in sph_mlp_apply

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2h __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (v_cvt_pk_bf16_f32), two at a time
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2h));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)(f2bf2(f, 0.f) & 0xffffu); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU(z) = z Phi(z) and GELU'(z) = Phi(z) + z phi(z), Phi the standard
// normal CDF.  Phi comes from the complementary error function,
// Phi(z) = erfc(-z / sqrt 2) / 2, with erfc(x) ~ t exp(-x^2 + P(t)),
// t = 1 / (1 + x / 2) for x >= 0: the Chebyshev-fitted approximation of
// Numerical Recipes (erfcc, fractional error below 1.2e-7 everywhere).  The
// negative tail is taken as erfc itself rather than 1 + erf(z / sqrt 2), so
// it keeps its relative accuracy; no branches.
__device__ __forceinline__ void normal_cdf_pdf(float z, float& Phi, float& e2) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.f));
    float p = fmaf(t, 0.17087277f, -0.82215223f);
    p = fmaf(t, p, 1.48851587f);
    p = fmaf(t, p, -1.13520398f);
    p = fmaf(t, p, 0.27886807f);
    p = fmaf(t, p, -0.18628806f);
    p = fmaf(t, p, 0.09678418f);
    p = fmaf(t, p, 0.37409196f);
    p = fmaf(t, p, 1.00002368f);
    p = fmaf(t, p, -1.26551223f);
    e2 = __expf(-x * x);                          // exp(-z^2 / 2)
    const float half_erfc = 0.5f * t * e2 * __expf(p);
    Phi = z >= 0.f ? 1.f - half_erfc : half_erfc;
}
__device__ __forceinline__ float gelu(float z) {
    float Phi, e2;
    normal_cdf_pdf(z, Phi, e2);
    return z * Phi;
}
__device__ __forceinline__ void gelu_and_grad(float z, float& g, float& gp) {
    float Phi, e2;
    normal_cdf_pdf(z, Phi, e2);
    g = z * Phi;
    gp = fmaf(z * e2, 0.39894228040143268f, Phi);
}

// ------------------------------------------------------------------ fused training pass
//
// One workgroup of four waves per CU walks 64-sample blocks of the batch
// (blocks blockIdx.x, blockIdx.x + gridDim.x, ...).  Each wave carries 16
// samples through the network with the unit index on the MFMA row axis and
// the sample on the column axis: the accumulator of one layer (lane (g, c)
// holds rows 4g..4g+3 of a 16-row tile for sample c) is then, unchanged, the
// B operand of the next layer's 16x16x16 MFMA, so activations never leave
// registers.  Weights sit in LDS as per-lane MFMA fragments.  Weight
// gradients contract over samples: their operands are staged in LDS as
// [unit][sample] BF16 arrays of the block, and each wave accumulates its
// quarter of dW1, dW2 and dW3 in MFMA accumulators across the blocks; bias
// gradients are summed per lane.  The workgroup writes one partial record,
// summed over workgroups in a fixed order by k_train_reduce.
//
// dW3 = dY^T bf16(H2) keeps dY in FP32: dY is split into three BF16 parts
// (hi + mid + lo reproduces the FP32 value) placed in separate B columns, so
// one MFMA tile yields the three partial products, added in FP32 at the end.

constexpr int TS = 16;            // samples per wave
constexpr int TWAVES = 4;         // waves per workgroup
constexpr int TB = TS * TWAVES;   // samples per block
constexpr int KS1 = 7;            // layer-1 K steps: feature columns 0..111 (100..111 are zero)
constexpr int NF1 = 16 * KS1;     // feature columns carried by dW1
constexpr int HT = NH / 16;       // hidden tiles
constexpr int SROW = TB + 8;      // staging row stride (BF16 elements)
// partial record of one workgroup (floats)
constexpr int PR_W1 = 0, PR_W2 = PR_W1 + NH * NF1, PR_W3 = PR_W2 + NH * NH, PR_B1 = PR_W3 + NOUT * NH,
              PR_B2 = PR_B1 + NH, PR_B3 = PR_B2 + NH, PR_LEN = ((PR_B3 + NOUT) + 63) & ~63;

struct TrainLds {
    bf16x4 w1f[HT][KS1][64];   // layer 1 A: W1b[16t + c][16ks + 4g + e]
    bf16x4 w2f[HT][HT][64];    // layer 2 A: W2b[16t + c][16ks + 4g + e]
    bf16x4 w2t[HT][HT][64];    // dH1 A:     W2b[16ks + 4g + e][16t + c]
    bf16x4 w3f[HT][64];        // layer 3 A: W3b[c][16ks + 4g + e] (rows c >= 3 zero)
    float w3v[NOUT][NH];       // bf16(W3) as FP32 for dH2 = dY W3b
    float b1[NH], b2[NH], b3[4];
    uint16_t xt[NF1][SROW];    // X^T of the block
    uint16_t h1t[NH][SROW];    // bf16(H1)^T, then bf16(dZ1)^T
    uint16_t s2t[NH][SROW];    // bf16(H2)^T, then bf16(dZ2)^T
    uint16_t dyt[16][SROW];    // dY parts: rows 0-2 hi, 3-5 mid, 6-8 lo, 9-15 zero
};
static_assert(sizeof(TrainLds) <= 160 * 1024, "LDS budget of the training pass");

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    return __builtin_bit_cast(bf16x4, make_uint2(f2bf2(a, b), f2bf2(c, d)));
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// z[t] = sum over ks of A[t][ks] b[ks] (t = 0 .. HT - 1), two tiles at a
// time: both tiles' weight fragments are read from LDS before their MFMAs,
// which alternate between the two accumulators, so neither an LDS read nor
// a dependent MFMA is waited on back to back (each tile keeps its order of
// accumulation over ks).
template <int KS>
__device__ __forceinline__ void tile_layer(const bf16x4 (&A)[HT][KS][64], int wl, const bf16x4* b, f32x4* z) {
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < HT; t += 2) {
        bf16x4 a0[KS], a1[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            a0[ks] = A[t][ks][wl];
            a1[ks] = A[t + 1][ks][wl];
        }
        f32x4 z0 = zero4, z1 = zero4;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            z0 = mfma16(a0[ks], b[ks], z0);
            z1 = mfma16(a1[ks], b[ks], z1);
        }
        z[t] = z0;
        z[t + 1] = z1;
    }
}

// forward-only LDS: the layer fragments and biases
struct FwdLds {
    bf16x4 w1f[HT][KS1][64];
    bf16x4 w2f[HT][HT][64];
    bf16x4 w3f[HT][64];
    float b1[NH], b2[NH], b3[4];
};

// weights -> LDS fragments (all WNT threads of the workgroup).  Each of a
// thread's fragments has a fixed slot; the thread loads a batch of them
// (unconditionally: padding columns read an in-range element and are zeroed
// after) before it packs and stores any, so the batch's global loads are in
// flight together rather than one round trip apiece.
constexpr int WNT = 256;
constexpr int W1_PER = HT * KS1 * 64 / WNT, W2_PER = HT * HT * 64 / WNT, W3_PER = HT * 64 / WNT;
static_assert(W1_PER * WNT == HT * KS1 * 64 && W2_PER * WNT == HT * HT * 64 && W3_PER * WNT == HT * 64, "whole trips");
template <bool TRAIN, class LDS>
__device__ void load_weights(LDS& L, const float* __restrict__ p) {
    const int tid = threadIdx.x;
    {
        float4 v[W1_PER];
#pragma unroll
        for (int k = 0; k < W1_PER; ++k) {
            const int i = tid + k * WNT;
            const int t = i / (KS1 * 64), ks = (i / 64) % KS1, ln = i % 64;
            const int row = 16 * t + (ln & 15), k0 = 16 * ks + 4 * (ln >> 4);
            v[k] = *reinterpret_cast<const float4*>(p + OFF_W1 + row * NIN + min(k0, NIN - 4));
        }
#pragma unroll
        for (int k = 0; k < W1_PER; ++k) {
            const int i = tid + k * WNT;
            const int t = i / (KS1 * 64), ks = (i / 64) % KS1, ln = i % 64;
            const bool pad = 16 * ks + 4 * (ln >> 4) >= NIN;
            L.w1f[t][ks][ln] = pad ? bf16x4{0, 0, 0, 0} : pack4(v[k].x, v[k].y, v[k].z, v[k].w);
        }
    }
    constexpr int W2_BATCH = 8;
    static_assert(W2_PER % W2_BATCH == 0, "whole batches");
#pragma unroll
    for (int k0 = 0; k0 < W2_PER; k0 += W2_BATCH) {
        float4 v[W2_BATCH], u[W2_BATCH];
#pragma unroll
        for (int k = 0; k < W2_BATCH; ++k) {
            const int i = tid + (k0 + k) * WNT;
            const int t = i / (HT * 64), ks = (i / 64) % HT, ln = i % 64;
            const int g = ln >> 4, c = ln & 15;
            v[k] = *reinterpret_cast<const float4*>(p + OFF_W2 + (16 * t + c) * NH + 16 * ks + 4 * g);
            if constexpr (TRAIN) {
                const float* q = p + OFF_W2 + (16 * ks + 4 * g) * NH + 16 * t + c;
                u[k] = float4{q[0], q[NH], q[2 * NH], q[3 * NH]};
            }
        }
#pragma unroll
        for (int k = 0; k < W2_BATCH; ++k) {
            const int i = tid + (k0 + k) * WNT;
            const int t = i / (HT * 64), ks = (i / 64) % HT, ln = i % 64;
            L.w2f[t][ks][ln] = pack4(v[k].x, v[k].y, v[k].z, v[k].w);
            if constexpr (TRAIN) L.w2t[t][ks][ln] = pack4(u[k].x, u[k].y, u[k].z, u[k].w);
        }
    }
    {
        float4 v[W3_PER];
#pragma unroll
        for (int k = 0; k < W3_PER; ++k) {
            const int i = tid + k * WNT;
            const int ks = i / 64, ln = i % 64, c = ln & 15;
            v[k] = *reinterpret_cast<const float4*>(p + OFF_W3 + min(c, NOUT - 1) * NH + 16 * ks + 4 * (ln >> 4));
        }
#pragma unroll
        for (int k = 0; k < W3_PER; ++k) {
            const int i = tid + k * WNT;
            const int ks = i / 64, ln = i % 64;
            L.w3f[ks][ln] = (ln & 15) >= NOUT ? bf16x4{0, 0, 0, 0} : pack4(v[k].x, v[k].y, v[k].z, v[k].w);
        }
    }
    static_assert(NH <= WNT, "one bias entry per thread");
    if (tid < NH) {
        L.b1[tid] = p[OFF_B1 + tid];
        L.b2[tid] = p[OFF_B2 + tid];
    }
    if (tid < 4) L.b3[tid] = tid < NOUT ? p[OFF_B3 + tid] : 0.f;
    if constexpr (TRAIN) {
#pragma unroll
        for (int k = 0; k < (NOUT * NH + WNT - 1) / WNT; ++k) {
            const int i = tid + k * WNT;
            if (i < NOUT * NH) L.w3v[i / NH][i % NH] = bf2f(f2bf(p[OFF_W3 + i]));
        }
        for (int i = tid; i < 16 * SROW; i += WNT) L.dyt[i / SROW][i % SROW] = 0;
    }
}

// Forward pass of n samples, 16 per wave (the layer chain of the training
// pass without its staging): Y FP32 [n][3].
__global__ void __launch_bounds__(256) k_forward_fused(int n, const float* __restrict__ params,
                                                       const uint16_t* __restrict__ X, float* __restrict__ Y) {
    __shared__ FwdLds L;
    load_weights<false>(L, params);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    const int nslab = (n + TS - 1) / TS;
    for (int sl = blockIdx.x * TWAVES + w; sl < nslab; sl += gridDim.x * TWAVES) {
        const int s = sl * TS + c;
        const bool valid = s < n;
        // an offset the compiler cannot prove loop-invariant: the weight
        // fragments are read from LDS at their use, not hoisted into registers
        int oz = 0;
        asm volatile("" : "+v"(oz));
        const int wl = lane + oz;
        bf16x4 xb[KS1];
        const uint16_t* xr = X + (valid ? (int64_t)s : 0) * FS + 4 * g;
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks)
            xb[ks] = valid ? *reinterpret_cast<const bf16x4*>(xr + 16 * ks) : bf16x4{0, 0, 0, 0};
        f32x4 z[HT];
        tile_layer<KS1>(L.w1f, wl, xb, z);
        bf16x4 h[HT];
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float4 bb = *reinterpret_cast<const float4*>(&L.b1[16 * t + 4 * g + oz]);
            h[t] = pack4(gelu(z[t][0] + bb.x), gelu(z[t][1] + bb.y), gelu(z[t][2] + bb.z), gelu(z[t][3] + bb.w));
        }
        tile_layer<HT>(L.w2f, wl, h, z);
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float4 bb = *reinterpret_cast<const float4*>(&L.b2[16 * t + 4 * g + oz]);
            h[t] = pack4(gelu(z[t][0] + bb.x), gelu(z[t][1] + bb.y), gelu(z[t][2] + bb.z), gelu(z[t][3] + bb.w));
        }
        f32x4 y = zero4;
#pragma unroll
        for (int ks = 0; ks < HT; ++ks) y = mfma16(L.w3f[ks][wl], h[ks], y);
        if (g == 0 && valid) {
#pragma unroll
            for (int o = 0; o < NOUT; ++o) Y[(int64_t)s * NOUT + o] = y[o] + L.b3[o];
        }
    }
}

// sum over the 16 lanes of a lane row (lanes with equal lane >> 4)
__device__ __forceinline__ float row16_sum(float v) {
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}
__device__ __forceinline__ double row16_sum(double v) {
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

// X: BF16 rows [nrows][FS]; sample b of the batch is row (idx ? idx[b] : b),
// an index outside [0, nrows) taken as the nearest valid row.
// part: [gridDim.x][PR_LEN] floats, lpart: [gridDim.x] doubles.
__global__ void __launch_bounds__(256) k_train_fused(int B, const float* __restrict__ params,
                                                     const uint16_t* __restrict__ X, int64_t nrows,
                                                     const int64_t* __restrict__ idx,
                                                     const float* __restrict__ T, float* __restrict__ part,
                                                     double* __restrict__ lpart) {
    __shared__ TrainLds L;
    load_weights<true>(L, params);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const float sc = 2.f / (3.f * (float)B);
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

    f32x4 aW1[2][KS1], aW2[2][HT], aW3[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int k = 0; k < KS1; ++k) aW1[a][k] = zero4;
#pragma unroll
        for (int k = 0; k < HT; ++k) aW2[a][k] = zero4;
        aW3[a] = zero4;
    }
    float db1[HT][4], db2[HT][4], db3[NOUT] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) db1[t][e] = db2[t][e] = 0.f;
    double lsum = 0.0;

    const int nblk = (B + TB - 1) / TB;
    const int col = w * TS + c;  // this lane's sample column in the block
    // the feature fragments of a block are loaded one block ahead
    auto sample_row = [&](int s) -> int64_t {
        int64_t r = s < B ? (idx ? idx[s] : (int64_t)s) : 0;
        return r < 0 ? 0 : (r >= nrows ? nrows - 1 : r);
    };
    auto load_x = [&](int s, int64_t r, bf16x4* xv) {
        const uint16_t* xr = X + r * FS + 4 * g;
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks)
            xv[ks] = s < B ? *reinterpret_cast<const bf16x4*>(xr + 16 * ks) : bf16x4{0, 0, 0, 0};
    };
    auto load_t = [&](int s, int64_t r, float* tv) {
#pragma unroll
        for (int o = 0; o < NOUT; ++o) tv[o] = (g == 0 && s < B) ? T[r * NOUT + o] : 0.f;
    };
    bf16x4 xn[KS1];
    float tn[NOUT];
    int64_t rown = 0;
    if (blockIdx.x < nblk) {
        rown = sample_row(blockIdx.x * TB + col);
        load_x(blockIdx.x * TB + col, rown, xn);
        load_t(blockIdx.x * TB + col, rown, tn);
    }
    for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int s = blk * TB + col;
        const bool valid = s < B;
        // an offset the compiler cannot prove loop-invariant: the weight
        // fragments are read from LDS at their use, not hoisted into registers
        int oz = 0;
        asm volatile("" : "+v"(oz));
        const int wl = lane + oz;
        bf16x4 xb[KS1];
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) xb[ks] = xn[ks];
        float tv[NOUT];
#pragma unroll
        for (int o = 0; o < NOUT; ++o) tv[o] = tn[o];
        if (blk + (int)gridDim.x < nblk) {
            const int sn = (blk + gridDim.x) * TB + col;
            rown = sample_row(sn);
            load_x(sn, rown, xn);
            load_t(sn, rown, tn);
        }
        // layer 1
        f32x4 z[HT];
        tile_layer<KS1>(L.w1f, wl, xb, z);
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks)
#pragma unroll
            for (int e = 0; e < 4; ++e) L.xt[16 * ks + 4 * g + e][col] = (uint16_t)xb[ks][e];
        bf16x4 h1[HT];
        float gp1[HT][4];
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float4 bb = *reinterpret_cast<const float4*>(&L.b1[16 * t + 4 * g + oz]);
            float hv[4];
            gelu_and_grad(z[t][0] + bb.x, hv[0], gp1[t][0]);
            gelu_and_grad(z[t][1] + bb.y, hv[1], gp1[t][1]);
            gelu_and_grad(z[t][2] + bb.z, hv[2], gp1[t][2]);
            gelu_and_grad(z[t][3] + bb.w, hv[3], gp1[t][3]);
            h1[t] = pack4(hv[0], hv[1], hv[2], hv[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) L.h1t[16 * t + 4 * g + e][col] = (uint16_t)h1[t][e];
        }
        // layer 2
        tile_layer<HT>(L.w2f, wl, h1, z);
        bf16x4 h2[HT];
        float gp2[HT][4];
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float4 bb = *reinterpret_cast<const float4*>(&L.b2[16 * t + 4 * g + oz]);
            float hv[4];
            gelu_and_grad(z[t][0] + bb.x, hv[0], gp2[t][0]);
            gelu_and_grad(z[t][1] + bb.y, hv[1], gp2[t][1]);
            gelu_and_grad(z[t][2] + bb.z, hv[2], gp2[t][2]);
            gelu_and_grad(z[t][3] + bb.w, hv[3], gp2[t][3]);
            h2[t] = pack4(hv[0], hv[1], hv[2], hv[3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) L.s2t[16 * t + 4 * g + e][col] = (uint16_t)h2[t][e];
        }
        // layer 3 (rows 0..2 of the 16-row tile are the outputs)
        f32x4 y = zero4;
#pragma unroll
        for (int ks = 0; ks < HT; ++ks) y = mfma16(L.w3f[ks][wl], h2[ks], y);
        // loss and dY = 2 (Y - T) / (3B); lanes of row 0 own the outputs of sample c
        float dyv[NOUT];
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            float d = 0.f;
            if (g == 0 && valid) d = (y[o] + L.b3[o]) - tv[o];
            dyv[o] = sc * d;
            lsum += (double)d * (double)d;
            db3[o] += dyv[o];
            if (g == 0) {
                uint16_t hi = f2bf(dyv[o]);
                float r1 = dyv[o] - bf2f(hi);
                uint16_t mid = f2bf(r1);
                float r2 = r1 - bf2f(mid);
                L.dyt[o][col] = hi;
                L.dyt[NOUT + o][col] = mid;
                L.dyt[2 * NOUT + o][col] = f2bf(r2);
            }
        }
        float dyc[NOUT];
#pragma unroll
        for (int o = 0; o < NOUT; ++o) dyc[o] = __shfl(dyv[o], c);
        // dZ2 = (dY bf16(W3)) * GELU'(Z2)
        bf16x4 dz2b[HT];
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float4 v0 = *reinterpret_cast<const float4*>(&L.w3v[0][16 * t + 4 * g + oz]);
            float4 v1 = *reinterpret_cast<const float4*>(&L.w3v[1][16 * t + 4 * g + oz]);
            float4 v2 = *reinterpret_cast<const float4*>(&L.w3v[2][16 * t + 4 * g + oz]);
            float wv[3][4] = {{v0.x, v0.y, v0.z, v0.w}, {v1.x, v1.y, v1.z, v1.w}, {v2.x, v2.y, v2.z, v2.w}};
            float dz[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float sacc = fmaf(dyc[0], wv[0][e], 0.f);
                sacc = fmaf(dyc[1], wv[1][e], sacc);
                sacc = fmaf(dyc[2], wv[2][e], sacc);
                dz[e] = sacc * gp2[t][e];
                db2[t][e] += dz[e];
            }
            dz2b[t] = pack4(dz[0], dz[1], dz[2], dz[3]);
        }
        __syncthreads();  // X^T, H1^T, H2^T and the dY parts of the block are staged
        // dW3^T tiles: rows j (this wave's two 16-row blocks), columns = dY parts
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int kk = 0; kk < TB / 16; ++kk) {
                bf16x4 av = *reinterpret_cast<const bf16x4*>(&L.s2t[16 * (2 * w + a) + c][16 * kk + 4 * g]);
                bf16x4 bv = *reinterpret_cast<const bf16x4*>(&L.dyt[c][16 * kk + 4 * g]);
                aW3[a] = mfma16(av, bv, aW3[a]);
            }
        __syncthreads();  // H2^T consumed
#pragma unroll
        for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) L.s2t[16 * t + 4 * g + e][col] = (uint16_t)dz2b[t][e];
        // dZ1 = (bf16(dZ2) bf16(W2)) * GELU'(Z1)
        tile_layer<HT>(L.w2t, wl, dz2b, z);
        bf16x4 dz1b[HT];
#pragma unroll
        for (int t = 0; t < HT; ++t) {
            float dz[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                dz[e] = z[t][e] * gp1[t][e];
                db1[t][e] += dz[e];
            }
            dz1b[t] = pack4(dz[0], dz[1], dz[2], dz[3]);
        }
        __syncthreads();  // dZ2^T staged
        // dW2 = bf16(dZ2)^T bf16(H1)
#pragma unroll
        for (int kk = 0; kk < TB / 16; ++kk) {
            bf16x4 av[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                av[a] = *reinterpret_cast<const bf16x4*>(&L.s2t[16 * (2 * w + a) + c][16 * kk + 4 * g]);
#pragma unroll
            for (int kb = 0; kb < HT; ++kb) {
                bf16x4 bv = *reinterpret_cast<const bf16x4*>(&L.h1t[16 * kb + c][16 * kk + 4 * g]);
#pragma unroll
                for (int a = 0; a < 2; ++a) aW2[a][kb] = mfma16(av[a], bv, aW2[a][kb]);
            }
        }
        __syncthreads();  // H1^T consumed
#pragma unroll
        for (int t = 0; t < HT; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) L.h1t[16 * t + 4 * g + e][col] = (uint16_t)dz1b[t][e];
        __syncthreads();  // dZ1^T staged
        // dW1 = bf16(dZ1)^T X
#pragma unroll
        for (int kk = 0; kk < TB / 16; ++kk) {
            bf16x4 av[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                av[a] = *reinterpret_cast<const bf16x4*>(&L.h1t[16 * (2 * w + a) + c][16 * kk + 4 * g]);
#pragma unroll
            for (int kb = 0; kb < KS1; ++kb) {
                bf16x4 bv = *reinterpret_cast<const bf16x4*>(&L.xt[16 * kb + c][16 * kk + 4 * g]);
#pragma unroll
                for (int a = 0; a < 2; ++a) aW1[a][kb] = mfma16(av[a], bv, aW1[a][kb]);
            }
        }
        __syncthreads();  // staging free for the next block
    }

    // partial record of the workgroup
    float* pr = part + (int64_t)blockIdx.x * PR_LEN;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 16 * (2 * w + a) + 4 * g + e;
#pragma unroll
            for (int kb = 0; kb < KS1; ++kb) pr[PR_W1 + j * NF1 + 16 * kb + c] = aW1[a][kb][e];
#pragma unroll
            for (int kb = 0; kb < HT; ++kb) pr[PR_W2 + j * NH + 16 * kb + c] = aW2[a][kb][e];
            // dW3[o][j] = parts hi + mid + lo (columns o, 3 + o, 6 + o)
            float v = aW3[a][e];
            float mid = __shfl(v, (lane + NOUT) & 63);
            float lo = __shfl(v, (lane + 2 * NOUT) & 63);
            if (c < NOUT) pr[PR_W3 + c * NH + j] = (lo + mid) + v;
        }
    // bias gradients and loss: lane rows, then waves in order
    float* red = reinterpret_cast<float*>(&L.xt[0][0]);  // [TWAVES][2 NH + 4]
    double* lred = reinterpret_cast<double*>(&L.h1t[0][0]);
#pragma unroll
    for (int t = 0; t < HT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float s1 = row16_sum(db1[t][e]);
            float s2 = row16_sum(db2[t][e]);
            if (c == 0) {
                red[w * (2 * NH + 4) + 16 * t + 4 * g + e] = s1;
                red[w * (2 * NH + 4) + NH + 16 * t + 4 * g + e] = s2;
            }
        }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        float s3 = row16_sum(db3[o]);
        if (lane == 0) red[w * (2 * NH + 4) + 2 * NH + o] = s3;
    }
    double ls = row16_sum(lsum);
    if (lane == 0) lred[w] = ls;
    __syncthreads();
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * NH + NOUT; i += blockDim.x) {
        float v = 0.f;
        for (int q = 0; q < TWAVES; ++q) v += red[q * (2 * NH + 4) + i];
        pr[PR_B1 + i] = v;  // b1, b2, b3 are contiguous in the record
    }
    if (tid == 0) {
        double v = 0.0;
        for (int q = 0; q < TWAVES; ++q) v += lred[q];
        lpart[blockIdx.x] = v;
    }
}

struct AdamArgs {
    float lr, beta1, beta2, eps, wd, bc1, bc2;  // bc = 1 - beta^step
};

// packed parameter index -> offset in a partial record
__device__ __forceinline__ int record_offset(int t) {
    if (t < OFF_B1) return PR_W1 + (t / NIN) * NF1 + t % NIN;
    if (t < OFF_W2) return PR_B1 + (t - OFF_B1);
    if (t < OFF_B2) return PR_W2 + (t - OFF_W2);
    if (t < OFF_W3) return PR_B2 + (t - OFF_B2);
    if (t < OFF_B3) return PR_W3 + (t - OFF_W3);
    return PR_B3 + (t - OFF_B3);
}

// Sum of the workgroup partials (records 0, 1, ... in four interleaved
// groups, the groups then added in order), AdamW update of the FP32 masters.
// Block: 64 parameters x 4 groups.  The last block also sums the loss.
__global__ void __launch_bounds__(256) k_train_reduce(int nrec, int B, const float* __restrict__ part,
                                                      const double* __restrict__ lpart, AdamArgs a,
                                                      float* __restrict__ p, float* __restrict__ m,
                                                      float* __restrict__ v, float* __restrict__ gout,
                                                      float* __restrict__ loss) {
    __shared__ float sg[4][64];
    __shared__ double sl[256];
    const int tid = threadIdx.x, q = tid >> 6, k = tid & 63;
    const int t = blockIdx.x * 64 + k;
    float acc = 0.f;
    if (t < NPARAM) {
        const int off = record_offset(t);
        const float* src = part + off;
        int r = q;
        for (; r + 60 < nrec; r += 64) {  // 16 loads in flight, added in record order
            float x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = src[(int64_t)(r + 4 * u) * PR_LEN];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += x[u];
        }
        for (; r < nrec; r += 4) acc += src[(int64_t)r * PR_LEN];
    }
    sg[q][k] = acc;
    if (loss && blockIdx.x == gridDim.x - 1) {
        double s = 0.0;
        for (int r = tid; r < nrec; r += 256) s += lpart[r];
        sl[tid] = s;
    }
    __syncthreads();
    if (loss && blockIdx.x == gridDim.x - 1) {
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) sl[tid] += sl[tid + h];
            __syncthreads();
        }
        if (tid == 0) *loss = (float)(sl[0] / (3.0 * (double)B));
    }
    if (q != 0 || t >= NPARAM) return;
    float gr = ((sg[0][k] + sg[1][k]) + sg[2][k]) + sg[3][k];
    if (gout) gout[t] = gr;
    if (a.lr == 0.f) return;  // gradient only
    float mm = a.beta1 * m[t] + (1.f - a.beta1) * gr;
    float vv = a.beta2 * v[t] + (1.f - a.beta2) * gr * gr;
    m[t] = mm;
    v[t] = vv;
    float mhat = mm / a.bc1;
    float vhat = vv / a.bc2;
    p[t] = p[t] * (1.f - a.lr * a.wd) - a.lr * mhat / (sqrtf(vhat) + a.eps);
}

// ------------------------------------------------------------------ features

__device__ __forceinline__ int fcoord(float x, float lo, float inv, int nc) {
    int c = (int)floorf((x - lo) * inv);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Neighbour selection for the features: keys are (|r_ij|^2 in FP64, j),
// compared lexicographically (a non-negative double orders like its bit
// pattern); the empty key is (UINT64_MAX, INT32_MAX).
constexpr uint64_t KEY_EMPTY = ~0ull;
constexpr int32_t J_EMPTY = 0x7fffffff;

__device__ __forceinline__ bool key_less(uint64_t ka, int32_t ja, uint64_t kb, int32_t jb) {
    return ka < kb || (ka == kb && ja < jb);
}

// compare-exchange with lane ^ m: keep the smaller key when take_min
__device__ __forceinline__ void key_cx(uint64_t& k, int32_t& j, int m, bool take_min) {
    const uint64_t ok = __shfl_xor(k, m, 64);
    const int32_t oj = __shfl_xor(j, m, 64);
    const bool other_less = key_less(ok, oj, k, j);
    if (other_less == take_min) {
        k = ok;
        j = oj;
    }
}

// ascending bitonic sort of one key per lane
__device__ __forceinline__ void key_sort64(uint64_t& k, int32_t& j, int lane) {
#pragma unroll
    for (int kk = 2; kk <= 64; kk <<= 1)
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            const bool asc = (lane & kk) == 0;
            const bool lower = (lane & jj) == 0;
            key_cx(k, j, jj, lower == asc);
        }
}

// A (ascending) := the 64 smallest of A and B (B unordered), ascending
__device__ __forceinline__ void key_merge(uint64_t& ak, int32_t& aj, uint64_t bk, int32_t bj, int lane) {
    key_sort64(bk, bj, lane);
    const uint64_t rk = __shfl(bk, 63 - lane, 64);  // B descending against A ascending:
    const int32_t rj = __shfl(bj, 63 - lane, 64);   // the lane-wise minima are the 64 smallest
    if (key_less(rk, rj, ak, aj)) {
        ak = rk;
        aj = rj;
    }
#pragma unroll
    for (int jj = 32; jj > 0; jj >>= 1) key_cx(ak, aj, jj, (lane & jj) == 0);  // bitonic -> ascending
}

// lane holding the r-th set bit (r from 0) of m
__device__ __forceinline__ int nth_set_lane(uint64_t m, int r) {
    int src = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int t = src + step;
        if (__popcll(m & ((1ull << t) - 1ull)) <= r) src = t;
    }
    return src;
}

// One wave per feature row (caller order, rows [r0, r0 + m)).  The particles
// are binned on cells at least h wide with linear (z, y, x) keys, so the
// candidates within 2h lie in 25 (z, y) rows of five cells, each row one
// contiguous slot range (a periodic x axis splits a row in two: lanes 25..49
// hold the wrapped pieces).  Lanes test 64 candidates at a time with the
// exact FP64 distance; those within 2h (j != i) are compacted by a ballot
// into a 64-slot batch, and each full batch is merged into the running 64
// nearest (bitonic sort and merge over lanes).  Lanes 0..31 then hold the 32
// nearest by (|r_ij|^2, j) and write the offsets (r_j - r_i)/h; then phi/h
// and grad phi; features rounded to BF16, columns 100.. zero.
constexpr int FEAT_WPB = 4;   // waves (rows) per block
constexpr int FEAT_DIV = 2;   // cells per 2h
constexpr int FEAT_ROWS = (2 * FEAT_DIV + 1) * (2 * FEAT_DIV + 1);

__global__ void __launch_bounds__(64 * FEAT_WPB) k_features(int32_t n, int32_t r0, int32_t m, BoxArgs b, double rc2,
                                                            float hinv, float cx, float cy, float cz, float R,
                                                            const int32_t* __restrict__ cell_start,
                                                            const float4* __restrict__ sorted,
                                                            const float4* __restrict__ pos4,
                                                            uint16_t* __restrict__ feat) {
    constexpr int NR = 2 * FEAT_ROWS;  // ranges: the rows, then their wrapped pieces
    const int lane = (int)(threadIdx.x & 63);
    const int32_t k = (int32_t)blockIdx.x * FEAT_WPB + (int32_t)(threadIdx.x >> 6);
    if (k >= m) return;  // the whole wave
    const int32_t i = r0 + k;
    const float4 p = pos4[i];
    // lane < NR: one slot range of the candidate block
    int32_t c0 = 0, cn = 0;
    if (lane < NR) {
        const int r = lane % FEAT_ROWS, part = lane / FEAT_ROWS;
        const int px = fcoord(p.x, b.lo[0], b.inv_cell[0], b.nc[0]);
        int y = fcoord(p.y, b.lo[1], b.inv_cell[1], b.nc[1]) + r % (2 * FEAT_DIV + 1) - FEAT_DIV;
        int z = fcoord(p.z, b.lo[2], b.inv_cell[2], b.nc[2]) + r / (2 * FEAT_DIV + 1) - FEAT_DIV;
        bool ok = true;
        if (b.periodic[1]) y = y < 0 ? y + b.nc[1] : (y >= b.nc[1] ? y - b.nc[1] : y);
        else ok = ok && y >= 0 && y < b.nc[1];
        if (b.periodic[2]) z = z < 0 ? z + b.nc[2] : (z >= b.nc[2] ? z - b.nc[2] : z);
        else ok = ok && z >= 0 && z < b.nc[2];
        if (ok) {
            const int nx = b.nc[0];
            const int32_t row = (z * b.nc[1] + y) * nx;
            int xa = px - FEAT_DIV, xb = px + FEAT_DIV, wa = 0, wb = -1;
            if (b.periodic[0]) {  // nx >= 2 FEAT_DIV + 1: at most one side wraps
                if (xa < 0) {
                    wa = xa + nx;
                    wb = nx - 1;
                    xa = 0;
                } else if (xb >= nx) {
                    wa = 0;
                    wb = xb - nx;
                    xb = nx - 1;
                }
            } else {
                xa = xa < 0 ? 0 : xa;
                xb = xb > nx - 1 ? nx - 1 : xb;
            }
            if (part == 1) {
                xa = wa;
                xb = wb;
            }
            if (xb >= xa) {
                c0 = cell_start[row + xa];
                cn = cell_start[row + xb + 1] - c0;
            }
        }
    }
    int32_t inc = cn;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    const int32_t exc = inc - cn;
    const int32_t total = __shfl(inc, NR - 1, 64);
    uint64_t ak = KEY_EMPTY, bk = KEY_EMPTY;
    int32_t aj = J_EMPTY, bj = J_EMPTY;
    int nb = 0;  // filled slots of the batch
    for (int32_t base = 0; base < total; base += 64) {
        const int32_t cidx = base + lane;
        int cc = 0;  // the last range whose block starts at or before cidx
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int mid = cc + step;
            const int32_t v = __shfl(exc, mid < NR ? mid : NR - 1, 64);
            if (mid < NR && v <= cidx) cc = mid;
        }
        const int32_t t = __shfl(c0, cc, 64) + (cidx - __shfl(exc, cc, 64));
        bool in = false;
        uint64_t key = KEY_EMPTY;
        int32_t j = J_EMPTY;
        if (cidx < total) {
            const float4 q = sorted[t];
            j = __float_as_int(q.w);
            double dx = (double)q.x - (double)p.x;
            double dy = (double)q.y - (double)p.y;
            double dz = (double)q.z - (double)p.z;
            if (b.periodic[0]) dx = dx > b.halfLd[0] ? dx - b.Ld[0] : (dx < -b.halfLd[0] ? dx + b.Ld[0] : dx);
            if (b.periodic[1]) dy = dy > b.halfLd[1] ? dy - b.Ld[1] : (dy < -b.halfLd[1] ? dy + b.Ld[1] : dy);
            if (b.periodic[2]) dz = dz > b.halfLd[2] ? dz - b.Ld[2] : (dz < -b.halfLd[2] ? dz + b.Ld[2] : dz);
            const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            in = j != i && d2 <= rc2;
            key = (uint64_t)__double_as_longlong(d2);
        }
        const uint64_t mk = __ballot(in);
        const int nin = (int)__popcll(mk);
        int taken = 0;
        while (taken < nin) {  // wave-uniform
            const int put = min(64 - nb, nin - taken);
            const int src = nth_set_lane(mk, min(max(lane - nb + taken, 0), nin - 1));
            const uint64_t sk = __shfl(key, src, 64);
            const int32_t sj = __shfl(j, src, 64);
            if (lane >= nb && lane < nb + put) {
                bk = sk;
                bj = sj;
            }
            nb += put;
            taken += put;
            if (nb == 64) {
                key_merge(ak, aj, bk, bj, lane);
                bk = KEY_EMPTY;
                bj = J_EMPTY;
                nb = 0;
            }
        }
    }
    if (nb > 0) key_merge(ak, aj, bk, bj, lane);
    uint16_t* f = feat + (int64_t)k * FS;
    if (lane < 32) {
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (aj != J_EMPTY) {
            const float4 q = pos4[aj];
            ox = min_image(q.x - p.x, b.L[0], b.halfL[0], b.periodic[0]) * hinv;
            oy = min_image(q.y - p.y, b.L[1], b.halfL[1], b.periodic[1]) * hinv;
            oz = min_image(q.z - p.z, b.L[2], b.halfL[2], b.periodic[2]) * hinv;
        }
        f[3 * lane + 0] = f2bf(ox);
        f[3 * lane + 1] = f2bf(oy);
        f[3 * lane + 2] = f2bf(oz);
    } else if (lane == 32) {
        const float ex = p.x - cx, ey = p.y - cy, ez = p.z - cz;
        const float rr = sqrtf(ex * ex + ey * ey + ez * ez);
        const float inv = rr > 0.f ? 1.f / rr : 0.f;
        f[96] = f2bf((rr - R) * hinv);
        f[97] = f2bf(ex * inv);
        f[98] = f2bf(ey * inv);
        f[99] = f2bf(ez * inv);
    } else if (lane < 32 + 1 + (FS - NIN)) {
        f[NIN + (lane - 33)] = 0;
    }
}

// r += h y, then bound to the sphere
__global__ void k_apply_disp(int32_t n, float h, float cx, float cy, float cz, float R, const float* __restrict__ y,
                             float* __restrict__ pos) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t nn = n;
    float x = pos[i] + h * y[(int64_t)i * NOUT + 0];
    float yy = pos[nn + i] + h * y[(int64_t)i * NOUT + 1];
    float z = pos[2 * nn + i] + h * y[(int64_t)i * NOUT + 2];
    float ex = x - cx, ey = yy - cy, ez = z - cz;
    float rr = sqrtf(ex * ex + ey * ey + ez * ez);
    float phi = rr - R;
    if (phi > 0.f && rr > 0.f) {
        float f = phi / rr;
        x -= f * ex;
        yy -= f * ey;
        z -= f * ez;
    }
    pos[i] = x;
    pos[nn + i] = yy;
    pos[2 * nn + i] = z;
}

// target (row-major [n][3]) = (to - from) / h, positions SoA [3][n]
__global__ void k_targets(int32_t n, float hinv, const float* __restrict__ from, const float* __restrict__ to,
                          float* __restrict__ target) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nn = n;
#pragma unroll
    for (int a = 0; a < NOUT; ++a) target[(int64_t)i * NOUT + a] = (to[a * nn + i] - from[a * nn + i]) * hinv;
}

// ------------------------------------------------------------------ host helpers

int forward_grid(sph_ctx* c, int32_t n) {
    if (c->num_cu <= 0) {
        int dev = 0, k = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&k, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            c->num_cu = k > 0 ? k : 1;
    }
    const int64_t waves = ((int64_t)n + TS - 1) / TS;
    const int64_t want = (waves + TWAVES - 1) / TWAVES, cap = 2 * (int64_t)(c->num_cu > 0 ? c->num_cu : 256);
    return (int)(want < cap ? want : cap);
}

// training-pass partials: one record per workgroup
struct TrainScratch {
    int nwg;
    float* part;
    double* lpart;
};

int train_scratch(sph_ctx* c, int32_t batch, TrainScratch* ts) {
    if (c->num_cu <= 0) {
        int dev = 0, n = 0;
        SPH_HIP(c, hipGetDevice(&dev));
        SPH_HIP(c, hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        c->num_cu = n > 0 ? n : 1;
    }
    const int nblk = (batch + TB - 1) / TB;
    ts->nwg = nblk < c->num_cu ? nblk : c->num_cu;
    const size_t pbytes = ((size_t)ts->nwg * PR_LEN * sizeof(float) + 255) & ~(size_t)255;
    SPH_HIP(c, c->tc.ensure(pbytes + (size_t)ts->nwg * sizeof(double)));
    ts->part = c->tc.as<float>();
    ts->lpart = reinterpret_cast<double*>(c->tc.as<char>() + pbytes);
    return SPH_OK;
}

void train_launch(sph_ctx* c, const TrainScratch& ts, const sph_adamw_params& ap, int64_t step, float* params,
                  float* m, float* v, int32_t batch, const uint16_t* feat, int64_t nrows, const int64_t* rows,
                  const float* target, float* loss, float* grad) {
    hipLaunchKernelGGL(k_train_fused, dim3(ts.nwg), dim3(256), 0, c->stream, batch, params, feat, nrows, rows, target,
                       ts.part, ts.lpart);
    bool update = ap.lr != 0.0;
    AdamArgs aa{};
    aa.lr = (float)ap.lr;
    aa.beta1 = (float)ap.beta1;
    aa.beta2 = (float)ap.beta2;
    aa.eps = (float)ap.eps;
    aa.wd = (float)ap.weight_decay;
    aa.bc1 = update ? (float)(1.0 - std::pow(ap.beta1, (double)step)) : 1.f;
    aa.bc2 = update ? (float)(1.0 - std::pow(ap.beta2, (double)step)) : 1.f;
    hipLaunchKernelGGL(k_train_reduce, dim3((NPARAM + 63) / 64), dim3(256), 0, c->stream, ts.nwg, batch, ts.part,
                       ts.lpart, aa, params, m, v, grad, loss);
}

}  // namespace

// ------------------------------------------------------------------ fixed workspace
// sph_mlp_train_step_noalloc keeps the training pass's per-workgroup partial
// records in this file-scope array instead of context scratch: room for
// NOALLOC_WG workgroups (PR_LEN floats each, 32.2 MB in all) and their FP64
// loss partials.  Each GPU holds its own copy for the life of the process;
// host code reaches it only through the address taken once per device by
// sph_mlp_noalloc_setup (the array's name is a host-side stand-in).
namespace {
constexpr int NOALLOC_WG = 256;
constexpr size_t NOALLOC_PART = ((size_t)NOALLOC_WG * PR_LEN * sizeof(float) + 255) & ~(size_t)255;
constexpr size_t NOALLOC_BYTES = NOALLOC_PART + (size_t)NOALLOC_WG * sizeof(double);
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_noalloc_err[NOALLOC_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Take the device address of the fixed workspace on the current device (once
// per device; later calls return at once).  Called by sph_ctx_create with the
// context's device current.  A failure is recorded for that device and
// reported by sph_mlp_train_step_noalloc; contexts work without it.
void sph_mlp_noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess && ptr) g_noalloc_ptr[device] = ptr;
    else g_noalloc_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

extern "C" {

int sph_mlp_train_step_noalloc(sph_ctx* c, const sph_adamw_params* ap, int64_t step, float* params, float* adam_m,
                               float* adam_v, int32_t batch, const uint16_t* feat, const float* target, float* loss,
                               float* grad) {
    if (!c) return SPH_ERR_ARG;
    if (!ap || !params || batch <= 0 || !feat || !target)
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_step_noalloc: bad arguments");
    const bool update = ap->lr != 0.0;
    if (update && (!adam_m || !adam_v || step < 1))
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_step_noalloc: moments and step >= 1 needed for an update");
    void* ws = nullptr;
    hipError_t werr = hipSuccess;
    if (c->device >= 0 && c->device < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        ws = g_noalloc_ptr[c->device];
        werr = g_noalloc_err[c->device];
    }
    if (!ws)
        return sph_fail(c, SPH_ERR_STATE, "sph_mlp_train_step_noalloc: fixed workspace unavailable on device %d (%s)",
                        c->device, werr == hipSuccess ? "not set up" : hipGetErrorString(werr));
    if (c->num_cu <= 0) {
        int n = 0;
        SPH_HIP(c, hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, c->device));
        c->num_cu = n > 0 ? n : 1;
    }
    // the same workgroup count as sph_mlp_train_step, hence the same sums
    const int nblk = (batch + TB - 1) / TB;
    TrainScratch ts;
    ts.nwg = nblk < c->num_cu ? nblk : c->num_cu;
    if (ts.nwg > NOALLOC_WG)
        return sph_fail(c, SPH_ERR_CAPACITY,
                        "sph_mlp_train_step_noalloc: %d workgroup records exceed the fixed workspace of %d", ts.nwg,
                        NOALLOC_WG);
    ts.part = static_cast<float*>(ws);
    ts.lpart = reinterpret_cast<double*>(static_cast<char*>(ws) + NOALLOC_PART);
    train_launch(c, ts, *ap, step, params, adam_m, adam_v, batch, feat, batch, nullptr, target, loss, grad);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"

extern "C" {

int sph_mlp_features(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, const float* pos,
                     uint16_t* feat) {
    if (!c) return SPH_ERR_ARG;
    if (c->dim != 3) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_features: 3-D only");
    if (!dom || !p) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_features: NULL domain or params");
    if (n < 0 || (n > 0 && (!pos || !feat))) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_features: bad arrays");
    sph_domain d = *dom;
    d.kernel = SPH_LAGUERRE_GAUSS;
    d.kappa = 2.0;
    int r = sph_bin_cells_grid(c, &d, n, pos, FEAT_DIV, true);
    if (r) return r;
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n, FEAT_WPB)), dim3(64 * FEAT_WPB), 0, c->stream, n, 0, n, c->box, c->rc2,
                       (float)(1.0 / d.h), (float)p->center[0], (float)p->center[1], (float)p->center[2],
                       (float)p->radius, c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->pos4.as<float4>(),
                       feat);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_mlp_forward(sph_ctx* c, const float* params, int32_t n, const uint16_t* feat, float* out) {
    if (!c) return SPH_ERR_ARG;
    if (n < 0 || !params || (n > 0 && (!feat || !out))) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_forward: bad arrays");
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_forward_fused, dim3(forward_grid(c, n)), dim3(256), 0, c->stream, n, params, feat, out);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_mlp_train_step(sph_ctx* c, const sph_adamw_params* ap, int64_t step, float* params, float* adam_m,
                       float* adam_v, int32_t batch, const uint16_t* feat, const float* target, float* loss,
                       float* grad) {
    if (!c) return SPH_ERR_ARG;
    if (!ap || !params || batch <= 0 || !feat || !target)
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_step: bad arguments");
    bool update = ap->lr != 0.0;
    if (update && (!adam_m || !adam_v || step < 1))
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_step: moments and step >= 1 needed for an update");
    TrainScratch ts;
    int r = train_scratch(c, batch, &ts);
    if (r) return r;
    train_launch(c, ts, *ap, step, params, adam_m, adam_v, batch, feat, batch, nullptr, target, loss, grad);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_mlp_train_epoch(sph_ctx* c, const sph_adamw_params* ap, int64_t step0, float* params, float* adam_m,
                        float* adam_v, int32_t batch, int32_t nbatch, int64_t nrows, const int64_t* rows,
                        const uint16_t* feat, const float* target, float* losses) {
    if (!c) return SPH_ERR_ARG;
    if (!ap || !params || batch <= 0 || nbatch < 0 || (nbatch > 0 && (nrows < 1 || !rows || !feat || !target)))
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_epoch: bad arguments");
    if (ap->lr == 0.0 || !adam_m || !adam_v || step0 < 1)
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_train_epoch: lr > 0, moments and step0 >= 1 needed");
    if (nbatch == 0) return SPH_OK;
    TrainScratch ts;
    int r = train_scratch(c, batch, &ts);
    if (r) return r;
    for (int32_t b = 0; b < nbatch; ++b)
        train_launch(c, ts, *ap, step0 + b, params, adam_m, adam_v, batch, feat, nrows, rows + (int64_t)b * batch,
                     target, losses ? losses + b : nullptr, nullptr);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_mlp_targets(sph_ctx* c, int32_t n, double h, const float* from, const float* to, float* target) {
    if (!c) return SPH_ERR_ARG;
    if (n < 0 || !(h > 0.0) || (n > 0 && (!from || !to || !target)))
        return sph_fail(c, SPH_ERR_ARG, "sph_mlp_targets: bad arguments");
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_targets, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, (float)(1.0 / h), from, to,
                       target);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_mlp_apply(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, float* pos,
                  const float* params) {
    if (!c) return SPH_ERR_ARG;
    if (c->dim != 3) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_apply: 3-D only");
    if (!dom || !p || !params || n < 0 || (n > 0 && !pos)) return sph_fail(c, SPH_ERR_ARG, "sph_mlp_apply: bad arguments");
    if (n == 0) return SPH_OK;
    sph_domain d = *dom;
    d.kernel = SPH_LAGUERRE_GAUSS;
    d.kappa = 2.0;
    int r = sph_bin_cells_grid(c, &d, n, pos, FEAT_DIV, true);
    if (r) return r;
    int rows = n < CHUNK ? n : CHUNK;
    SPH_HIP(c, c->ua.ensure((size_t)rows * FS * sizeof(uint16_t)));  // feature chunk
    SPH_HIP(c, c->ub.ensure((size_t)n * NOUT * sizeof(float)));      // displacements
    for (int32_t r0 = 0; r0 < n; r0 += CHUNK) {
        int m = n - r0 < CHUNK ? n - r0 : CHUNK;
        hipLaunchKernelGGL(k_features, dim3(grid_for(m, FEAT_WPB)), dim3(64 * FEAT_WPB), 0, c->stream, n, r0, m, c->box,
                           c->rc2,
                           (float)(1.0 / d.h), (float)p->center[0], (float)p->center[1], (float)p->center[2],
                           (float)p->radius, c->cell_start.as<int32_t>(), c->sorted.as<float4>(),
                           c->pos4.as<float4>(), c->ua.as<uint16_t>());
        hipLaunchKernelGGL(k_forward_fused, dim3(forward_grid(c, m)), dim3(256), 0, c->stream, m, params,
                           c->ua.as<uint16_t>(), c->ub.as<float>() + (int64_t)r0 * NOUT);
    }
    hipLaunchKernelGGL(k_apply_disp, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, (float)d.h,
                       (float)p->center[0], (float)p->center[1], (float)p->center[2], (float)p->radius,
                       c->ub.as<float>(), pos);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
