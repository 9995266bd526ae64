// sph_mlp.hip -- the learned warm start of the relaxation: neighbour-offset
// features, a 100-128-128-3 GELU network on BF16 MFMA tiles with FP32
// accumulation, its training step (backward + AdamW on FP32 masters), and
// its application to a relaxing configuration.
//
// Rounding points (shared with the oracle): weights, layer inputs and the
// backward GEMM operands are rounded to BF16 (nearest-even); bias, GELU,
// loss and optimizer arithmetic are FP32.
//
// GEMMs use v_mfma_f32_16x16x16_bf16: a 256-thread block computes a 64x64
// tile of C = A B (four waves, each 2x2 MFMA tiles), A and B read as BF16
// through (row, column) strides so transposed operands need no copies, with
// the K range optionally split across blocks (partials reduced in a fixed
// order, so results are deterministic).
#include "sph_internal.h"

namespace {

constexpr int NIN = 100, NH = 128, NOUT = 3;
constexpr int FS = SPH_MLP_FEAT_STRIDE;  // feature row stride (zero padded)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == SPH_MLP_NPARAMS, "parameter count");
constexpr int CHUNK = 1 << 18;  // samples per forward pass in sph_mlp_forward / sph_mlp_apply

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    uint32_t r = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + r) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ GEMM

enum { EPI_STORE = 0, EPI_GELU = 1, EPI_BWD_GELU = 2 };

struct Epi {
    float* C;              // FP32 output [M][ldc] (EPI_STORE: + blockIdx.z * split_stride)
    int ldc;
    int64_t split_stride;
    const float* bias;     // per column (EPI_STORE, EPI_GELU), nullable
    float* Z;              // EPI_GELU: pre-activation out (nullable)
    uint16_t* Hb;          // EPI_GELU: bf16(GELU(z)); EPI_BWD_GELU: bf16(dz)
    int ldh;
    const float* Zin;      // EPI_BWD_GELU: saved pre-activation [M][ldz]
    int ldz;
};

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kchunk, const uint16_t* __restrict__ A,
                                              int64_t sam, int64_t sak, const uint16_t* __restrict__ B, int64_t sbk,
                                              int64_t sbn, Epi ep) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + 32 * (w >> 1);
    const int n0 = blockIdx.y * 64 + 32 * (w & 1);
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int li = lane & 15, lk = 4 * (lane >> 4);
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = kb; k < ke; k += 16) {
        bf16x4 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            int row = m0 + 16 * t + li;
            int kk = k + lk;
            if (sak == 1 && row < M && kk + 3 < ke) {
                av[t] = *reinterpret_cast<const bf16x4*>(A + row * sam + kk);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    av[t][e] = (row < M && kk + e < ke) ? (short)A[row * sam + (int64_t)(kk + e) * sak] : (short)0;
            }
            int colb = n0 + 16 * t + li;
            if (sbk == 1 && colb < N && kk + 3 < ke) {
                bv[t] = *reinterpret_cast<const bf16x4*>(B + colb * sbn + kk);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    bv[t][e] = (colb < N && kk + e < ke) ? (short)B[(int64_t)(kk + e) * sbk + colb * sbn] : (short)0;
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    // accumulator element e of tile (a, b): row m0+16a+4(lane/16)+e, column n0+16b+lane%16
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int col = n0 + 16 * b + li;
            if (col >= N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int row = m0 + 16 * a + lk + e;
                if (row >= M) continue;
                float v = acc[a][b][e];
                if (EPI == EPI_STORE) {
                    if (ep.bias) v += ep.bias[col];
                    ep.C[(int64_t)blockIdx.z * ep.split_stride + (int64_t)row * ep.ldc + col] = v;
                } else if (EPI == EPI_GELU) {
                    float z = v + ep.bias[col];
                    if (ep.Z) ep.Z[(int64_t)row * ep.ldc + col] = z;
                    ep.Hb[(int64_t)row * ep.ldh + col] = f2bf(gelu(z));
                } else {
                    float dz = v * gelu_grad(ep.Zin[(int64_t)row * ep.ldz + col]);
                    ep.C[(int64_t)row * ep.ldc + col] = dz;
                    ep.Hb[(int64_t)row * ep.ldh + col] = f2bf(dz);
                }
            }
        }
}

// ------------------------------------------------------------------ small kernels

// masters -> BF16 copies: W1b [128][FS] (K padded with zeros), W2b [128][128], W3b [16][128] (rows >= 3 zero)
__global__ void k_cast_weights(const float* __restrict__ p, uint16_t* __restrict__ W1b, uint16_t* __restrict__ W2b,
                               uint16_t* __restrict__ W3b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < NH * FS) {
        int r = t / FS, k = t % FS;
        W1b[t] = k < NIN ? f2bf(p[OFF_W1 + r * NIN + k]) : (uint16_t)0;
    }
    if (t < NH * NH) W2b[t] = f2bf(p[OFF_W2 + t]);
    if (t < 16 * NH) {
        int r = t / NH;
        W3b[t] = r < NOUT ? f2bf(p[OFF_W3 + t]) : (uint16_t)0;
    }
}

// dY = 2 (Y - T) / (3B); per-block partial sums of (Y - T)^2 in FP64
__global__ void k_loss_dy(int B, const float* __restrict__ Y, int ldy, const float* __restrict__ T,
                          float* __restrict__ dY, double* __restrict__ part) {
    __shared__ double s[256];
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (b < B) {
        float sc = 2.f / (3.f * (float)B);
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            float d = Y[(int64_t)b * ldy + o] - T[(int64_t)b * NOUT + o];
            dY[(int64_t)b * NOUT + o] = sc * d;
            acc += (double)d * d;
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_loss_final(int nb, int B, const double* __restrict__ part, float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    for (int k = 0; k < nb; ++k) acc += part[k];
    *loss = (float)(acc / (3.0 * (double)B));
}

// dZ2 = (dY W3b) * GELU'(Z2): FP32 and BF16 copies
__global__ void k_dz2(int B, const float* __restrict__ dY, const uint16_t* __restrict__ W3b,
                      const float* __restrict__ Z2, float* __restrict__ dZ2, uint16_t* __restrict__ dZ2b) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * NH) return;
    int64_t b = t / NH;
    int j = (int)(t % NH);
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < NOUT; ++o) s = fmaf(dY[b * NOUT + o], bf2f(W3b[o * NH + j]), s);
    float dz = s * gelu_grad(Z2[t]);
    dZ2[t] = dz;
    dZ2b[t] = f2bf(dz);
}

// partial column sums of X [rows][ld] over row chunks: part[chunk][col], col < ncols
__global__ void k_colsum_part(int rows, int ncols, const float* __restrict__ X, int ld, int rows_per_chunk,
                              float* __restrict__ part) {
    int col = threadIdx.x;
    if (col >= ncols) return;
    int r0 = blockIdx.x * rows_per_chunk;
    int r1 = min(rows, r0 + rows_per_chunk);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += X[(int64_t)r * ld + col];
    part[(int64_t)blockIdx.x * ncols + col] = s;
}

// dW3 partials: part[chunk][o][j] = sum_{b in chunk} dY[b][o] H2b[b][j]
__global__ void k_dw3_part(int B, const float* __restrict__ dY, const uint16_t* __restrict__ H2b, int rows_per_chunk,
                           float* __restrict__ part) {
    int j = threadIdx.x;  // 128 threads
    int r0 = blockIdx.x * rows_per_chunk;
    int r1 = min(B, r0 + rows_per_chunk);
    float s[NOUT] = {0.f, 0.f, 0.f};
    for (int r = r0; r < r1; ++r) {
        float hv = bf2f(H2b[(int64_t)r * NH + j]);
#pragma unroll
        for (int o = 0; o < NOUT; ++o) s[o] = fmaf(dY[(int64_t)r * NOUT + o], hv, s[o]);
    }
#pragma unroll
    for (int o = 0; o < NOUT; ++o) part[((int64_t)blockIdx.x * NOUT + o) * NH + j] = s[o];
}

// out[e] = sum_s part[s][e] in order s = 0, 1, ...
__global__ void k_reduce_parts(int nparts, int64_t E, const float* __restrict__ part, float* __restrict__ out) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    float s = 0.f;
    for (int k = 0; k < nparts; ++k) s += part[(int64_t)k * E + e];
    out[e] = s;
}

struct GradPtrs {
    const float *dW1, *db1, *dW2, *db2, *dW3, *db3;  // dW1 [128][FS]
};

struct AdamArgs {
    float lr, beta1, beta2, eps, wd, bc1, bc2;  // bc = 1 - beta^step
};

// gather the packed gradient, AdamW update of the FP32 masters
__global__ void k_adamw(GradPtrs g, AdamArgs a, float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                        float* __restrict__ gout) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    float gr;
    if (t < OFF_B1) gr = g.dW1[(t / NIN) * FS + t % NIN];
    else if (t < OFF_W2) gr = g.db1[t - OFF_B1];
    else if (t < OFF_B2) gr = g.dW2[t - OFF_W2];
    else if (t < OFF_W3) gr = g.db2[t - OFF_B2];
    else if (t < OFF_B3) gr = g.dW3[t - OFF_W3];
    else gr = g.db3[t - OFF_B3];
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

// One thread per particle (caller order, rows [r0, r0 + m)): the 32 nearest
// j != i within 2h by (|r_ij|^2 in FP64, j) (an unrolled insertion network in
// registers), then offsets (r_j - r_i)/h, phi/h and grad phi, rounded to BF16.
__global__ void __launch_bounds__(128) k_features(int32_t n, int32_t r0, int32_t m, BoxArgs b, double rc2, float hinv,
                                                  float cx, float cy, float cz, float R,
                                                  const int32_t* __restrict__ cell_start,
                                                  const float4* __restrict__ sorted, const float4* __restrict__ pos4,
                                                  uint16_t* __restrict__ feat) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    int32_t i = r0 + k;
    float4 p = pos4[i];
    double kd[32];
    int kj[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) {
        kd[s] = 1e300;
        kj[s] = 0x7fffffff;
    }
    int cxi = fcoord(p.x, b.lo[0], b.inv_cell[0], b.nc[0]);
    int cyi = fcoord(p.y, b.lo[1], b.inv_cell[1], b.nc[1]);
    int czi = fcoord(p.z, b.lo[2], b.inv_cell[2], b.nc[2]);
    for (int oz = -1; oz <= 1; ++oz) {
        int z = czi + oz;
        if (b.periodic[2]) z = z < 0 ? z + b.nc[2] : (z >= b.nc[2] ? z - b.nc[2] : z);
        else if (z < 0 || z >= b.nc[2]) continue;
        for (int oy = -1; oy <= 1; ++oy) {
            int y = cyi + oy;
            if (b.periodic[1]) y = y < 0 ? y + b.nc[1] : (y >= b.nc[1] ? y - b.nc[1] : y);
            else if (y < 0 || y >= b.nc[1]) continue;
            for (int ox = -1; ox <= 1; ++ox) {
                int x = cxi + ox;
                if (b.periodic[0]) x = x < 0 ? x + b.nc[0] : (x >= b.nc[0] ? x - b.nc[0] : x);
                else if (x < 0 || x >= b.nc[0]) continue;
                int32_t key = cell_key(b, x, y, z);
                int t1 = cell_start[key + 1];
                for (int t = cell_start[key]; t < t1; ++t) {
                    float4 q = sorted[t];
                    int j = __float_as_int(q.w);
                    if (j == i) continue;
                    double dx = (double)q.x - (double)p.x;
                    double dy = (double)q.y - (double)p.y;
                    double dz = (double)q.z - (double)p.z;
                    if (b.periodic[0]) dx = dx > b.halfLd[0] ? dx - b.Ld[0] : (dx < -b.halfLd[0] ? dx + b.Ld[0] : dx);
                    if (b.periodic[1]) dy = dy > b.halfLd[1] ? dy - b.Ld[1] : (dy < -b.halfLd[1] ? dy + b.Ld[1] : dy);
                    if (b.periodic[2]) dz = dz > b.halfLd[2] ? dz - b.Ld[2] : (dz < -b.halfLd[2] ? dz + b.Ld[2] : dz);
                    double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                    if (d2 > rc2) continue;
                    if (d2 > kd[31] || (d2 == kd[31] && j > kj[31])) continue;
                    double cd = d2;
                    int cj = j;
#pragma unroll
                    for (int s = 0; s < 32; ++s) {
                        bool lt = cd < kd[s] || (cd == kd[s] && cj < kj[s]);
                        double td = lt ? kd[s] : cd;
                        int tj = lt ? kj[s] : cj;
                        kd[s] = lt ? cd : kd[s];
                        kj[s] = lt ? cj : kj[s];
                        cd = td;
                        cj = tj;
                    }
                }
            }
        }
    }
    uint16_t* f = feat + (int64_t)k * FS;
#pragma unroll
    for (int s = 0; s < 32; ++s) {
        float ox = 0.f, oy = 0.f, oz2 = 0.f;
        if (kj[s] != 0x7fffffff) {
            float4 q = pos4[kj[s]];
            ox = min_image(q.x - p.x, b.L[0], b.halfL[0], b.periodic[0]) * hinv;
            oy = min_image(q.y - p.y, b.L[1], b.halfL[1], b.periodic[1]) * hinv;
            oz2 = min_image(q.z - p.z, b.L[2], b.halfL[2], b.periodic[2]) * hinv;
        }
        f[3 * s + 0] = f2bf(ox);
        f[3 * s + 1] = f2bf(oy);
        f[3 * s + 2] = f2bf(oz2);
    }
    float ex = p.x - cx, ey = p.y - cy, ez = p.z - cz;
    float rr = sqrtf(ex * ex + ey * ey + ez * ez);
    float inv = rr > 0.f ? 1.f / rr : 0.f;
    f[96] = f2bf((rr - R) * hinv);
    f[97] = f2bf(ex * inv);
    f[98] = f2bf(ey * inv);
    f[99] = f2bf(ez * inv);
    for (int s = NIN; s < FS; ++s) f[s] = 0;
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

// ------------------------------------------------------------------ host helpers

struct MlpScratch {
    uint16_t *W1b, *W2b, *W3b;
    float *Z1, *Z2, *Y, *dY, *dZ1, *dZ2;
    uint16_t *H1b, *H2b, *dZ1b, *dZ2b;
    float *part, *gW1, *gW2, *gW3, *gb1, *gb2, *gb3;
    double* lpart;
};

// carve the context's MLP scratch for up to `rows` samples
int mlp_scratch(sph_ctx* c, int64_t rows, bool train, MlpScratch* s) {
    const int64_t nchunks = 256;
    size_t need = 0;
    auto add = [&](size_t bytes) {
        size_t off = need;
        need += (bytes + 255) & ~(size_t)255;
        return off;
    };
    size_t oW1 = add(NH * FS * 2), oW2 = add(NH * NH * 2), oW3 = add(16 * NH * 2);
    size_t oZ1 = train ? add(rows * NH * 4) : 0, oZ2 = train ? add(rows * NH * 4) : 0;
    size_t oY = add(rows * NOUT * 4 + 64), odY = train ? add(rows * NOUT * 4) : 0;
    size_t odZ1 = train ? add(rows * NH * 4) : 0, odZ2 = train ? add(rows * NH * 4) : 0;
    size_t oH1 = add(rows * NH * 2), oH2 = add(rows * NH * 2);
    size_t odZ1b = train ? add(rows * NH * 2) : 0, odZ2b = train ? add(rows * NH * 2) : 0;
    size_t opart = train ? add((size_t)nchunks * NH * FS * 4) : 0;
    size_t ogW1 = train ? add(NH * FS * 4) : 0, ogW2 = train ? add(NH * NH * 4) : 0, ogW3 = train ? add(NOUT * NH * 4) : 0;
    size_t ogb1 = train ? add(NH * 4) : 0, ogb2 = train ? add(NH * 4) : 0, ogb3 = train ? add(64) : 0;
    size_t olp = add((rows / 256 + 2) * 8);
    SPH_HIP(c, c->tc.ensure(need));
    char* base = c->tc.as<char>();
    s->W1b = (uint16_t*)(base + oW1);
    s->W2b = (uint16_t*)(base + oW2);
    s->W3b = (uint16_t*)(base + oW3);
    s->Z1 = train ? (float*)(base + oZ1) : nullptr;
    s->Z2 = train ? (float*)(base + oZ2) : nullptr;
    s->Y = (float*)(base + oY);
    s->dY = train ? (float*)(base + odY) : nullptr;
    s->dZ1 = train ? (float*)(base + odZ1) : nullptr;
    s->dZ2 = train ? (float*)(base + odZ2) : nullptr;
    s->H1b = (uint16_t*)(base + oH1);
    s->H2b = (uint16_t*)(base + oH2);
    s->dZ1b = train ? (uint16_t*)(base + odZ1b) : nullptr;
    s->dZ2b = train ? (uint16_t*)(base + odZ2b) : nullptr;
    s->part = train ? (float*)(base + opart) : nullptr;
    s->gW1 = train ? (float*)(base + ogW1) : nullptr;
    s->gW2 = train ? (float*)(base + ogW2) : nullptr;
    s->gW3 = train ? (float*)(base + ogW3) : nullptr;
    s->gb1 = train ? (float*)(base + ogb1) : nullptr;
    s->gb2 = train ? (float*)(base + ogb2) : nullptr;
    s->gb3 = train ? (float*)(base + ogb3) : nullptr;
    s->lpart = (double*)(base + olp);
    return SPH_OK;
}

template <int EPI>
void gemm(sph_ctx* c, int M, int N, int K, int splits, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
          int64_t sbk, int64_t sbn, const Epi& ep) {
    int kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + 15) & ~15;
    int nz = (K + kchunk - 1) / kchunk;
    dim3 grid((M + 63) / 64, (N + 63) / 64, nz < 1 ? 1 : nz);
    hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, c->stream, M, N, K, kchunk, A, sam, sak, B, sbk, sbn, ep);
}

// forward of `rows` samples: X (bf16 [rows][FS]) -> Y (FP32 [rows][3]);
// with training buffers also keeps Z1, Z2.
void forward(sph_ctx* c, const MlpScratch& s, const float* params, int rows, const uint16_t* X, float* Yout,
             bool keep) {
    Epi e1{};
    e1.bias = params + OFF_B1;
    e1.Z = keep ? s.Z1 : nullptr;
    e1.ldc = NH;
    e1.Hb = s.H1b;
    e1.ldh = NH;
    gemm<EPI_GELU>(c, rows, NH, FS, 1, X, FS, 1, s.W1b, 1, FS, e1);
    Epi e2 = e1;
    e2.bias = params + OFF_B2;
    e2.Z = keep ? s.Z2 : nullptr;
    e2.Hb = s.H2b;
    gemm<EPI_GELU>(c, rows, NH, NH, 1, s.H1b, NH, 1, s.W2b, 1, NH, e2);
    Epi e3{};
    e3.C = Yout;
    e3.ldc = NOUT;
    e3.bias = params + OFF_B3;
    gemm<EPI_STORE>(c, rows, NOUT, NH, 1, s.H2b, NH, 1, s.W3b, 1, NH, e3);
}

}  // namespace

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
    int r = sph_bin_cells(c, &d, n, pos);
    if (r) return r;
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_features, dim3(grid_for(n, 128)), dim3(128), 0, c->stream, n, 0, n, c->box, c->rc2,
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
    int rows = n < CHUNK ? n : CHUNK;
    MlpScratch s;
    int r = mlp_scratch(c, rows, false, &s);
    if (r) return r;
    hipLaunchKernelGGL(k_cast_weights, dim3(grid_for(NH * FS, 256)), dim3(256), 0, c->stream, params, s.W1b, s.W2b,
                       s.W3b);
    for (int32_t r0 = 0; r0 < n; r0 += CHUNK) {
        int m = n - r0 < CHUNK ? n - r0 : CHUNK;
        forward(c, s, params, m, feat + (int64_t)r0 * FS, out + (int64_t)r0 * NOUT, false);
    }
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
    MlpScratch s;
    int r = mlp_scratch(c, batch, true, &s);
    if (r) return r;
    const int B = batch;
    hipLaunchKernelGGL(k_cast_weights, dim3(grid_for(NH * FS, 256)), dim3(256), 0, c->stream, params, s.W1b, s.W2b,
                       s.W3b);
    forward(c, s, params, B, feat, s.Y, true);
    int nb = (int)grid_for(B, 256);
    hipLaunchKernelGGL(k_loss_dy, dim3(nb), dim3(256), 0, c->stream, B, s.Y, NOUT, target, s.dY, s.lpart);
    if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1), 0, c->stream, nb, B, s.lpart, loss);
    // layer 3
    const int nchunk = 256;
    int rpc = (B + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_dw3_part, dim3(nchunk), dim3(NH), 0, c->stream, B, s.dY, s.H2b, rpc, s.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(NOUT * NH, 256)), dim3(256), 0, c->stream, nchunk,
                       (int64_t)NOUT * NH, s.part, s.gW3);
    hipLaunchKernelGGL(k_colsum_part, dim3(nchunk), dim3(64), 0, c->stream, B, NOUT, s.dY, NOUT, rpc, s.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, c->stream, nchunk, (int64_t)NOUT, s.part, s.gb3);
    // layer 2
    hipLaunchKernelGGL(k_dz2, dim3(grid_for((int64_t)B * NH, 256)), dim3(256), 0, c->stream, B, s.dY, s.W3b, s.Z2,
                       s.dZ2, s.dZ2b);
    Epi ew{};
    ew.C = s.part;
    ew.ldc = NH;
    ew.split_stride = (int64_t)NH * NH;
    gemm<EPI_STORE>(c, NH, NH, B, nchunk, s.dZ2b, 1, NH, s.H1b, NH, 1, ew);  // dW2 = dZ2^T H1
    int kchunk = (((B + nchunk - 1) / nchunk) + 15) & ~15;
    int nsplit = (B + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(NH * NH, 256)), dim3(256), 0, c->stream, nsplit,
                       (int64_t)NH * NH, s.part, s.gW2);
    hipLaunchKernelGGL(k_colsum_part, dim3(nchunk), dim3(NH), 0, c->stream, B, NH, s.dZ2, NH, rpc, s.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(NH), 0, c->stream, nchunk, (int64_t)NH, s.part, s.gb2);
    // layer 1
    Epi eb{};
    eb.C = s.dZ1;
    eb.ldc = NH;
    eb.Hb = s.dZ1b;
    eb.ldh = NH;
    eb.Zin = s.Z1;
    eb.ldz = NH;
    gemm<EPI_BWD_GELU>(c, B, NH, NH, 1, s.dZ2b, NH, 1, s.W2b, NH, 1, eb);  // dH1 = dZ2 W2, times GELU'(Z1)
    Epi e1{};
    e1.C = s.part;
    e1.ldc = FS;
    e1.split_stride = (int64_t)NH * FS;
    gemm<EPI_STORE>(c, NH, FS, B, nchunk, s.dZ1b, 1, NH, feat, FS, 1, e1);  // dW1 = dZ1^T X
    hipLaunchKernelGGL(k_reduce_parts, dim3(grid_for(NH * FS, 256)), dim3(256), 0, c->stream, nsplit,
                       (int64_t)NH * FS, s.part, s.gW1);
    hipLaunchKernelGGL(k_colsum_part, dim3(nchunk), dim3(NH), 0, c->stream, B, NH, s.dZ1, NH, rpc, s.part);
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(NH), 0, c->stream, nchunk, (int64_t)NH, s.part, s.gb1);
    // gradient and update
    GradPtrs gp{s.gW1, s.gb1, s.gW2, s.gb2, s.gW3, s.gb3};
    AdamArgs aa{};
    aa.lr = (float)ap->lr;
    aa.beta1 = (float)ap->beta1;
    aa.beta2 = (float)ap->beta2;
    aa.eps = (float)ap->eps;
    aa.wd = (float)ap->weight_decay;
    aa.bc1 = update ? (float)(1.0 - std::pow(ap->beta1, (double)step)) : 1.f;
    aa.bc2 = update ? (float)(1.0 - std::pow(ap->beta2, (double)step)) : 1.f;
    hipLaunchKernelGGL(k_adamw, dim3(grid_for(NPARAM, 256)), dim3(256), 0, c->stream, gp, aa, params, adam_m, adam_v,
                       grad);
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
    int r = sph_bin_cells(c, &d, n, pos);
    if (r) return r;
    int rows = n < CHUNK ? n : CHUNK;
    MlpScratch s;
    r = mlp_scratch(c, rows, false, &s);
    if (r) return r;
    SPH_HIP(c, c->ua.ensure((size_t)rows * FS * sizeof(uint16_t)));  // feature chunk
    SPH_HIP(c, c->ub.ensure((size_t)n * NOUT * sizeof(float)));      // displacements
    hipLaunchKernelGGL(k_cast_weights, dim3(grid_for(NH * FS, 256)), dim3(256), 0, c->stream, params, s.W1b, s.W2b,
                       s.W3b);
    for (int32_t r0 = 0; r0 < n; r0 += CHUNK) {
        int m = n - r0 < CHUNK ? n - r0 : CHUNK;
        hipLaunchKernelGGL(k_features, dim3(grid_for(m, 128)), dim3(128), 0, c->stream, n, r0, m, c->box, c->rc2,
                           (float)(1.0 / d.h), (float)p->center[0], (float)p->center[1], (float)p->center[2],
                           (float)p->radius, c->cell_start.as<int32_t>(), c->sorted.as<float4>(),
                           c->pos4.as<float4>(), c->ua.as<uint16_t>());
        forward(c, s, params, m, c->ua.as<uint16_t>(), c->ub.as<float>() + (int64_t)r0 * NOUT, false);
    }
    hipLaunchKernelGGL(k_apply_disp, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, n, (float)d.h,
                       (float)p->center[0], (float)p->center[1], (float)p->center[2], (float)p->radius,
                       c->ub.as<float>(), pos);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
