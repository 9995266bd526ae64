// sph_pairs.hip -- per-particle neighbour loops on the bound configuration:
// kernel summation, the correction matrix B_i (Eq. 9) with its FP64
// inversion, the cached geometry records, and the corrected gradient.
//
// Kernel sum and correction matrix: each cell-sorted (Morton) slot is taken
// by a group of LN lanes that split its row (fixed-stride ELL rows when the
// padding budget allows them, else the sorted CSR row), read one packed
// (x, y, z, V) record per neighbour through 32-bit offsets with the next
// record in flight, and merge their compensated (Kahan) partial sums with a
// TwoSum butterfly; the periodic wrap is applied only by waves holding a
// particle within a cut-off of a periodic face.  Blocks are remapped so each
// XCD works on one contiguous range of slots.  Caller-indexed inputs are
// gathered once into sorted order and outputs written back at the caller
// index.
#include "sph_internal.h"

namespace {

constexpr int BLK = 256;

template <int DIM>
__device__ __forceinline__ void pair_d(const float4& pi, const float4& pj, const BoxArgs& b, float d[3]) {
    d[0] = min_image(pi.x - pj.x, b.L[0], b.halfL[0], b.periodic[0]);
    d[1] = min_image(pi.y - pj.y, b.L[1], b.halfL[1], b.periodic[1]);
    d[2] = DIM == 3 ? min_image(pi.z - pj.z, b.L[2], b.halfL[2], b.periodic[2]) : 0.f;
}

// dst[s] = src[caller index of slot s]
__global__ void k_to_sorted(int32_t n, const float4* __restrict__ sorted, const float* __restrict__ src,
                            float* __restrict__ dst) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    dst[s] = src[__float_as_int(sorted[s].w)];
}

__device__ __forceinline__ int32_t slot_id() {
    return xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * (int32_t)blockDim.x + (int32_t)threadIdx.x;
}

// rec[s] = (x, y, z, V) of sorted slot s (z = 0 in 2-D)
__global__ void k_pair_rec(int32_t n, const float4* __restrict__ sorted, const float* __restrict__ vol,
                           float4* __restrict__ rec) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 p = sorted[s];
    rec[s] = make_float4(p.x, p.y, p.z, vol[__float_as_int(p.w)]);
}

// separation r_i - r_j of a pair (wrapped on periodic axes when WRAP)
template <int DIM, bool WRAP>
__device__ __forceinline__ void pair_sep(const Wrap& w, const float4& pi, const float4& pj, float d[3]) {
    d[0] = pi.x - pj.x;
    d[1] = pi.y - pj.y;
    d[2] = DIM == 3 ? pi.z - pj.z : 0.f;
    if (WRAP) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) d[a] = wrap1(d[a], w.L[a], w.invL[a]);
    }
}

// Kernel sum sum_j W_ij V_j (self term included).  ELL rows are padded with
// the slot itself; those entries (and only those: rows hold no self entry)
// are skipped.
template <int DIM, bool ELL, int LN>
__global__ void __launch_bounds__(BLK) k_kernel_sum(int32_t n, KernelConsts kc, Wrap w,
                                                    const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    int32_t S, const float4* __restrict__ rec,
                                                    const float4* __restrict__ sorted, float* __restrict__ out) {
    const int64_t tt = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;
    const int32_t i = (int32_t)(tt / LN);
    const int sub = (int)(tt % LN);
    if (i >= n) return;
    const float4 pi = ld32(rec, (uint32_t)i);
    const bool wrap = wave_needs_wrap(w, pi);
    Kahan acc;
    acc.init(sub == 0 ? kernel_W(kc, 0.f) * pi.w : 0.f);
    int64_t k, e, stride;
    row_range<ELL, LN>(i, sub, n, rp, S, k, e, stride);
    int32_t j = k < e ? col[k] : i;
    float4 pj = ld32(rec, (uint32_t)j);
    int32_t jn = k + stride < e ? col[k + stride] : i;
    while (k < e) {
        const float4 pn = ld32(rec, (uint32_t)jn);
        const int32_t jc = j;
        j = jn;
        jn = k + 2 * stride < e ? col[k + 2 * stride] : i;
        k += stride;
        float d[3];
        if (wrap) pair_sep<DIM, true>(w, pi, pj, d);
        else pair_sep<DIM, false>(w, pi, pj, d);
        const float r2 = fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2]));
        const float q = __builtin_amdgcn_sqrtf(r2) * kc.hinv;
        acc.add(jc != i ? kernel_W(kc, q) * pj.w : 0.f);
        pj = pn;
    }
    const float v = group_sum<LN>(acc);
    if (sub == 0) out[__float_as_int(sorted[i].w)] = v;
}

// FP64 inverse of the symmetric matrix given by its upper triangle
// (2-D: m00 m01 m11; 3-D: m00 m01 m02 m11 m12 m22) by adjugate / det.
// Returns false for the degenerate case |det| < 1e-10 |tr/d|^d.
template <int DIM>
__device__ __forceinline__ bool inv_sym(const double* m, double* inv) {
    if (DIM == 2) {
        double det = m[0] * m[2] - m[1] * m[1];
        double tr = 0.5 * (m[0] + m[2]);
        if (!(fabs(det) >= 1e-10 * tr * tr) || tr == 0.0) return false;
        double id = 1.0 / det;
        inv[0] = m[2] * id;
        inv[1] = -m[1] * id;
        inv[2] = m[0] * id;
        return true;
    }
    double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    // cofactors of [[a b c][b d e][c e f]]
    double A = d * f - e * e;
    double B = c * e - b * f;
    double C = b * e - c * d;
    double D = a * f - c * c;
    double E = b * c - a * e;
    double F = a * d - b * b;
    double det = a * A + b * B + c * C;
    double tr = (a + d + f) / 3.0;
    if (!(fabs(det) >= 1e-10 * fabs(tr * tr * tr)) || tr == 0.0) return false;
    double id = 1.0 / det;
    inv[0] = A * id;
    inv[1] = B * id;
    inv[2] = C * id;
    inv[3] = D * id;
    inv[4] = E * id;
    inv[5] = F * id;
    return true;
}

template <int DIM>
__device__ __forceinline__ void store_geo(int32_t i, const float4& p, float V, const float* Bu,
                                          float4* __restrict__ geo0, float4* __restrict__ geo1,
                                          float2* __restrict__ geo2) {
    if (DIM == 2) {
        geo0[i] = make_float4(p.x, p.y, V, Bu[0]);
        reinterpret_cast<float2*>(geo1)[i] = make_float2(Bu[1], Bu[2]);
    } else {
        geo0[i] = make_float4(p.x, p.y, p.z, V);
        geo1[i] = make_float4(Bu[0], Bu[1], Bu[2], Bu[3]);
        geo2[i] = make_float2(Bu[4], Bu[5]);
    }
}

// Correction matrix B_i = -(sum_j V_j (r_i - r_j) (x) grad W_ij)^-1 (Eq. 9),
// the sum in FP32 Kahan partials merged to FP64, inverted in FP64; a
// degenerate sum (fewer than DIM independent neighbour directions) gives the
// identity and is counted.  Also writes the cached geometry records.
template <int DIM, bool ELL, int LN>
__global__ void __launch_bounds__(BLK) k_correction(int32_t n, KernelConsts kc, Wrap w,
                                                    const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    int32_t S, const float4* __restrict__ rec,
                                                    const float4* __restrict__ sorted, float* __restrict__ Bout,
                                                    double* __restrict__ B64, float4* __restrict__ geo0,
                                                    float4* __restrict__ geo1, float2* __restrict__ geo2,
                                                    int32_t* __restrict__ ndeg) {
    constexpr int NU = DIM == 2 ? 3 : 6;
    const int64_t tt = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;
    const int32_t s = (int32_t)(tt / LN);
    const int sub = (int)(tt % LN);
    if (s >= n) return;
    const float4 pi = ld32(rec, (uint32_t)s);
    const bool wrap = wave_needs_wrap(w, pi);
    Kahan M[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) M[u].init();
    int64_t k, e, stride;
    row_range<ELL, LN>(s, sub, n, rp, S, k, e, stride);
    int32_t j = k < e ? col[k] : s;
    float4 pj = ld32(rec, (uint32_t)j);
    int32_t jn = k + stride < e ? col[k + stride] : s;
    while (k < e) {
        const float4 pn = ld32(rec, (uint32_t)jn);
        jn = k + 2 * stride < e ? col[k + 2 * stride] : s;
        k += stride;
        float d[3];
        if (wrap) pair_sep<DIM, true>(w, pi, pj, d);
        else pair_sep<DIM, false>(w, pi, pj, d);
        const float r2 = fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2]));
        const float q = __builtin_amdgcn_sqrtf(r2) * kc.hinv;
        const float wt = kernel_F(kc, q) * pj.w;  // grad W = F d;  r (x) grad W V = F V d d^T (zero for d = 0)
        if (DIM == 2) {
            M[0].add(wt * d[0] * d[0]);
            M[1].add(wt * d[0] * d[1]);
            M[2].add(wt * d[1] * d[1]);
        } else {
            M[0].add(wt * d[0] * d[0]);
            M[1].add(wt * d[0] * d[1]);
            M[2].add(wt * d[0] * d[2]);
            M[3].add(wt * d[1] * d[1]);
            M[4].add(wt * d[1] * d[2]);
            M[5].add(wt * d[2] * d[2]);
        }
        pj = pn;
    }
    double m[NU], inv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) m[u] = group_sum64<LN>(M[u]);
    if (sub != 0) return;
    const float4 ps = sorted[s];
    const int32_t i = __float_as_int(ps.w);
    double Bd[NU];
    if (inv_sym<DIM>(m, inv)) {
#pragma unroll
        for (int u = 0; u < NU; ++u) Bd[u] = -inv[u];
    } else {
        atomicAdd(ndeg, 1);
        if (DIM == 2) {
            Bd[0] = 1.0; Bd[1] = 0.0; Bd[2] = 1.0;
        } else {
            Bd[0] = 1.0; Bd[1] = 0.0; Bd[2] = 0.0; Bd[3] = 1.0; Bd[4] = 0.0; Bd[5] = 1.0;
        }
    }
    float Bu[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) Bu[u] = (float)Bd[u];
    // full matrices (upper triangle mirrored)
    if (DIM == 2) {
        const int idx[4] = {0, 1, 1, 2};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            Bout[(int64_t)i * 4 + t] = Bu[idx[t]];
            if (B64) B64[(int64_t)i * 4 + t] = Bd[idx[t]];
        }
    } else {
        const int idx[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            Bout[(int64_t)i * 9 + t] = Bu[idx[t]];
            if (B64) B64[(int64_t)i * 9 + t] = Bd[idx[t]];
        }
    }
    store_geo<DIM>(s, pi, pi.w, Bu, geo0, geo1, geo2);
}

template <int DIM>
__global__ void k_set_geo(int32_t n, const float4* __restrict__ sorted, const float* __restrict__ vol,
                          const float* __restrict__ B, float4* __restrict__ geo0, float4* __restrict__ geo1,
                          float2* __restrict__ geo2) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float4 ps = sorted[s];
    int32_t i = __float_as_int(ps.w);
    float Bu[6];
    if (DIM == 2) {
        const float* m = B + (int64_t)i * 4;
        Bu[0] = m[0]; Bu[1] = m[1]; Bu[2] = m[3];
    } else {
        const float* m = B + (int64_t)i * 9;
        Bu[0] = m[0]; Bu[1] = m[1]; Bu[2] = m[2]; Bu[3] = m[4]; Bu[4] = m[5]; Bu[5] = m[8];
    }
    store_geo<DIM>(s, ps, vol[i], Bu, geo0, geo1, geo2);
}

// Unpack the upper triangle of B_i from the geometry records.
template <int DIM>
__device__ __forceinline__ void load_B(int32_t i, const float4* __restrict__ geo0, const float4* __restrict__ geo1,
                                       const float2* __restrict__ geo2, float4& g0, float* Bu) {
    g0 = geo0[i];
    if (DIM == 2) {
        float2 t = reinterpret_cast<const float2*>(geo1)[i];
        Bu[0] = g0.w; Bu[1] = t.x; Bu[2] = t.y;
    } else {
        float4 t = geo1[i];
        float2 u = geo2[i];
        Bu[0] = t.x; Bu[1] = t.y; Bu[2] = t.z; Bu[3] = t.w; Bu[4] = u.x; Bu[5] = u.y;
    }
}

template <int DIM>
__global__ void k_gradient(int32_t n, BoxArgs b, float hinv, float cF, const int64_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col, const float4* __restrict__ geo0,
                           const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                           const float4* __restrict__ sorted, const float* __restrict__ f,
                           float* __restrict__ grad) {
    int32_t s = slot_id();
    if (s >= n) return;
    float4 gi;
    float Bu[6];
    load_B<DIM>(s, geo0, geo1, geo2, gi, Bu);
    int32_t i = __float_as_int(sorted[s].w);
    float fi = f[s];
    Kahan acc[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc[a].init();
    int64_t e = row_ptr[s + 1];
    for (int64_t k = row_ptr[s]; k < e; ++k) {
        int32_t t = col[k];
        float4 gj = geo0[t];
        float d[3];
        pair_d<DIM>(gi, gj, b, d);
        float r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        float q = sqrtf(r2) * hinv;
        float Vj = DIM == 2 ? gj.z : gj.w;
        float w = wendland_F(q, cF) * Vj * (f[t] - fi);
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc[a].add(w * d[a]);
    }
    float v[3] = {acc[0].value(), acc[1].value(), DIM == 3 ? acc[DIM - 1].value() : 0.f};
    if (DIM == 2) {
        grad[i] = Bu[0] * v[0] + Bu[1] * v[1];
        grad[(int64_t)n + i] = Bu[1] * v[0] + Bu[2] * v[1];
    } else {
        grad[i] = Bu[0] * v[0] + Bu[1] * v[1] + Bu[2] * v[2];
        grad[(int64_t)n + i] = Bu[1] * v[0] + Bu[3] * v[1] + Bu[4] * v[2];
        grad[2 * (int64_t)n + i] = Bu[2] * v[0] + Bu[4] * v[1] + Bu[5] * v[2];
    }
}

int to_sorted(sph_ctx* c, const float* src, DevBuf& dst) {
    SPH_HIP(c, dst.ensure((size_t)(c->n > 0 ? c->n : 1) * sizeof(float)));
    if (c->n > 0) {
        hipLaunchKernelGGL(k_to_sorted, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                           c->sorted.as<float4>(), src, dst.as<float>());
        SPH_LAUNCH_CHECK(c);
    }
    return SPH_OK;
}

// Lanes per slot for the kernel-sum and correction loops: the most (up to 8)
// that leave each lane at least eight row entries (measured on the 3-D
// Taylor-Green lattice: rows of 32 entries run fastest on 4 lanes, rows of
// 80 on 8; 2-D rows of 12 on one).  Override SPH_PAIR_LANES = 1, 2, 4 or 8.
int pair_lanes(const sph_ctx* c) {
    if (const char* e = getenv("SPH_PAIR_LANES")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8) return v;
    }
    const double avg = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    int L = 1;
    while (L < 8 && avg / (2 * L) >= 8.0) L <<= 1;
    return L;
}

// Packed records in c->svol and the row layout; the launch helper calls
// go(kernel, ell) with the kernel instantiated for the lane count.
int prepare_pair_loop(sph_ctx* c, const float* vol) {
    if (c->n >= (1 << 28))  // records are addressed through 32-bit byte offsets
        return sph_fail(c, SPH_ERR_CAPACITY, "pair loops: at most 2^28 - 1 particles");
    SPH_HIP(c, c->svol.ensure((size_t)c->n * sizeof(float4)));
    hipLaunchKernelGGL(k_pair_rec, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, c->sorted.as<float4>(),
                       vol, c->svol.as<float4>());
    return sph_ell_prepare(c);
}

template <int DIM, int LN>
void launch_kernel_sum_l(sph_ctx* c, const KernelConsts& kc, float* out) {
    const bool ell = c->ell_state == 1;
    const Wrap w = make_wrap(c);
    dim3 g(grid_for((int64_t)c->n * LN, BLK)), b(BLK);
    if (ell)
        hipLaunchKernelGGL((k_kernel_sum<DIM, true, LN>), g, b, 0, c->stream, c->n, kc, w, c->rp_s.as<int64_t>(),
                           c->colE.as<int32_t>(), c->ell_S, c->svol.as<float4>(), c->sorted.as<float4>(), out);
    else
        hipLaunchKernelGGL((k_kernel_sum<DIM, false, LN>), g, b, 0, c->stream, c->n, kc, w, c->rp_s.as<int64_t>(),
                           c->col_s.as<int32_t>(), 0, c->svol.as<float4>(), c->sorted.as<float4>(), out);
}

template <int DIM>
void launch_kernel_sum(sph_ctx* c, const KernelConsts& kc, float* out) {
    switch (pair_lanes(c)) {
        case 1: launch_kernel_sum_l<DIM, 1>(c, kc, out); break;
        case 2: launch_kernel_sum_l<DIM, 2>(c, kc, out); break;
        case 4: launch_kernel_sum_l<DIM, 4>(c, kc, out); break;
        default: launch_kernel_sum_l<DIM, 8>(c, kc, out); break;
    }
}

template <int DIM, int LN>
void launch_correction_l(sph_ctx* c, const KernelConsts& kc, float* B, double* B64, int32_t* ndeg) {
    const bool ell = c->ell_state == 1;
    const Wrap w = make_wrap(c);
    dim3 g(grid_for((int64_t)c->n * LN, BLK)), b(BLK);
    if (ell)
        hipLaunchKernelGGL((k_correction<DIM, true, LN>), g, b, 0, c->stream, c->n, kc, w, c->rp_s.as<int64_t>(),
                           c->colE.as<int32_t>(), c->ell_S, c->svol.as<float4>(), c->sorted.as<float4>(), B, B64,
                           c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), ndeg);
    else
        hipLaunchKernelGGL((k_correction<DIM, false, LN>), g, b, 0, c->stream, c->n, kc, w, c->rp_s.as<int64_t>(),
                           c->col_s.as<int32_t>(), 0, c->svol.as<float4>(), c->sorted.as<float4>(), B, B64,
                           c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), ndeg);
}

template <int DIM>
void launch_correction(sph_ctx* c, const KernelConsts& kc, float* B, double* B64, int32_t* ndeg) {
    switch (pair_lanes(c)) {
        case 1: launch_correction_l<DIM, 1>(c, kc, B, B64, ndeg); break;
        case 2: launch_correction_l<DIM, 2>(c, kc, B, B64, ndeg); break;
        case 4: launch_correction_l<DIM, 4>(c, kc, B, B64, ndeg); break;
        default: launch_correction_l<DIM, 8>(c, kc, B, B64, ndeg); break;
    }
}

int ensure_geo(sph_ctx* c) {
    int64_t nn = c->n > 0 ? c->n : 1;
    SPH_HIP(c, c->geo0.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->geo1.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->geo2.ensure(nn * sizeof(float2)));
    return SPH_OK;
}

}  // namespace

extern "C" {

int sph_kernel_sum(sph_ctx* c, const float* vol, float* out) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound) return sph_fail(c, SPH_ERR_STATE, "sph_kernel_sum: no configuration bound");
    if (c->n > 0 && (!vol || !out)) return sph_fail(c, SPH_ERR_ARG, "sph_kernel_sum: NULL array");
    if (c->n == 0) return SPH_OK;
    int r = prepare_pair_loop(c, vol);
    if (r) return r;
    KernelConsts kc = make_kernel_consts(c->dom.kernel, c->dim, c->dom.h);
    if (c->dim == 2) launch_kernel_sum<2>(c, kc, out);
    else launch_kernel_sum<3>(c, kc, out);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_correction_B(sph_ctx* c, const float* vol, float* B, double* B64, int32_t* n_degenerate) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound) return sph_fail(c, SPH_ERR_STATE, "sph_correction_B: no configuration bound");
    if (c->n > 0 && (!vol || !B)) return sph_fail(c, SPH_ERR_ARG, "sph_correction_B: NULL array");
    int r = ensure_geo(c);
    if (r) return r;
    // row layout first: its set-up uses the context counter too
    if (c->n > 0) {
        r = prepare_pair_loop(c, vol);
        if (r) return r;
    }
    SPH_HIP(c, c->counter.ensure(64));
    int32_t* ndeg = c->counter.as<int32_t>();
    SPH_HIP(c, hipMemsetAsync(ndeg, 0, sizeof(int32_t), c->stream));
    if (c->n > 0) {
        KernelConsts kc = make_kernel_consts(c->dom.kernel, c->dim, c->dom.h);
        if (c->dim == 2) launch_correction<2>(c, kc, B, B64, ndeg);
        else launch_correction<3>(c, kc, B, B64, ndeg);
        SPH_LAUNCH_CHECK(c);
    }
    if (n_degenerate) {
        SPH_HIP(c, hipMemcpyAsync(n_degenerate, ndeg, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        SPH_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->geo_valid = true;
    ++c->geo_gen;
    return SPH_OK;
}

int sph_set_correction(sph_ctx* c, const float* vol, const float* B) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound) return sph_fail(c, SPH_ERR_STATE, "sph_set_correction: no configuration bound");
    if (c->n > 0 && (!vol || !B)) return sph_fail(c, SPH_ERR_ARG, "sph_set_correction: NULL array");
    int r = ensure_geo(c);
    if (r) return r;
    if (c->n > 0) {
        if (c->dim == 2)
            hipLaunchKernelGGL(k_set_geo<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                               c->sorted.as<float4>(), vol, B, c->geo0.as<float4>(), c->geo1.as<float4>(),
                               c->geo2.as<float2>());
        else
            hipLaunchKernelGGL(k_set_geo<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                               c->sorted.as<float4>(), vol, B, c->geo0.as<float4>(), c->geo1.as<float4>(),
                               c->geo2.as<float2>());
        SPH_LAUNCH_CHECK(c);
    }
    c->geo_valid = true;
    ++c->geo_gen;
    return SPH_OK;
}

int sph_gradient(sph_ctx* c, const float* f, float* grad) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound || !c->geo_valid)
        return sph_fail(c, SPH_ERR_STATE, "sph_gradient: needs a bound configuration and a cached correction");
    if (c->dom.kernel != SPH_WENDLAND) return sph_fail(c, SPH_ERR_ARG, "sph_gradient: Wendland kernel only");
    if (c->n > 0 && (!f || !grad)) return sph_fail(c, SPH_ERR_ARG, "sph_gradient: NULL array");
    if (c->n == 0) return SPH_OK;
    int r = to_sorted(c, f, c->sfield);
    if (r) return r;
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, c->dim, c->dom.h);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_gradient<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, c->box, kc.hinv,
                           kc.cF, c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), c->geo0.as<float4>(),
                           c->geo1.as<float4>(), c->geo2.as<float2>(), c->sorted.as<float4>(), c->sfield.as<float>(),
                           grad);
    else
        hipLaunchKernelGGL(k_gradient<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, c->box, kc.hinv,
                           kc.cF, c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), c->geo0.as<float4>(),
                           c->geo1.as<float4>(), c->geo2.as<float2>(), c->sorted.as<float4>(), c->sfield.as<float>(),
                           grad);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
