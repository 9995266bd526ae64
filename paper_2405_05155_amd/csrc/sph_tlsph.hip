// sph_tlsph.hip -- total Lagrangian SPH (Sec. 3.2) on the reference
// configuration bound in the context: deformation rate (Eq. 32), PK1
// stress (Eq. 30 or compressible neo-Hookean), stress divergence (Eq. 31),
// and kick-drift-kick stepping.  3-D.
//
// Per step two neighbour loops:
//   A: gather half-step velocities -> dF/dt, F update, position drift,
//      P(F) and the per-particle record A_i = P_i B0_i^T (9 floats);
//   B: gather A_j -> acceleration, velocity kick.
// The stress is evaluated from H = F - I so that small strains keep FP32
// resolution (no I - C^{-1} or ln J cancellation).  Velocity, acceleration,
// A records, F and the current positions live in cell-sorted (Morton) order
// for the duration of a call (gathered from and scattered back to the
// caller's arrays at its start and end).
#include "sph_internal.h"

#include <cstdlib>
#include <cstring>

namespace {

constexpr int BLK = 256;

struct TlArgs {
    float lam, G, inv_rho0, dt, half_dt;
    float hinv, cF;
    float nhh;  // -hinv / 2
    int model;
};

__device__ __forceinline__ void pk1_from_H(const float* H, const TlArgs& t, float* P) {
    // 2E = H + H^T + H^T H
    float E2[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = H[r * 3 + c] + H[c * 3 + r];
#pragma unroll
            for (int k = 0; k < 3; ++k) s += H[k * 3 + r] * H[k * 3 + c];
            E2[r * 3 + c] = s;
        }
    float S[9];
    if (t.model == 1) {
        // St. Venant-Kirchhoff (Eq. 30): S = lambda tr(E) I + 2 G E
        float trE = 0.5f * (E2[0] + E2[4] + E2[8]);
#pragma unroll
        for (int k = 0; k < 9; ++k) S[k] = t.G * E2[k];
        S[0] += t.lam * trE;
        S[4] += t.lam * trE;
        S[8] += t.lam * trE;
    } else {
        // neo-Hookean: S = G C^{-1} (C - I) + lambda ln J C^{-1}, C = I + 2E
        float C[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) C[k] = E2[k];
        C[0] += 1.f;
        C[4] += 1.f;
        C[8] += 1.f;
        float A0 = C[4] * C[8] - C[5] * C[7];
        float A1 = C[2] * C[7] - C[1] * C[8];
        float A2 = C[1] * C[5] - C[2] * C[4];
        float A3 = C[5] * C[6] - C[3] * C[8];
        float A4 = C[0] * C[8] - C[2] * C[6];
        float A5 = C[2] * C[3] - C[0] * C[5];
        float A6 = C[3] * C[7] - C[4] * C[6];
        float A7 = C[1] * C[6] - C[0] * C[7];
        float A8 = C[0] * C[4] - C[1] * C[3];
        float detC = C[0] * A0 + C[1] * A3 + C[2] * A6;
        float idet = 1.f / detC;
        float Ci[9] = {A0 * idet, A1 * idet, A2 * idet, A3 * idet, A4 * idet,
                       A5 * idet, A6 * idet, A7 * idet, A8 * idet};
        // J - 1 = det(I + H) - 1 = tr H + (tr^2 H - tr H^2)/2 + det H
        float trH = H[0] + H[4] + H[8];
        float trH2 = 0.f;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) trH2 += H[r * 3 + c] * H[c * 3 + r];
        float detH = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                     H[2] * (H[3] * H[7] - H[4] * H[6]);
        float Jm1 = trH + 0.5f * (trH * trH - trH2) + detH;
        float lnJ = log1pf(Jm1);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float s = 0.f;
#pragma unroll
                for (int k = 0; k < 3; ++k) s += Ci[r * 3 + k] * E2[k * 3 + c];
                S[r * 3 + c] = t.G * s + t.lam * lnJ * Ci[r * 3 + c];
            }
    }
    // P = F S = S + H S
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = S[r * 3 + c];
#pragma unroll
            for (int k = 0; k < 3; ++k) s += H[r * 3 + k] * S[k * 3 + c];
            P[r * 3 + c] = s;
        }
}

__device__ __forceinline__ void load_B3(int32_t i, const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                        float* B) {
    const float4 t = ld32(geo1, (uint32_t)i);
    const float2 u = ld32(geo2, (uint32_t)i);
    B[0] = t.x; B[1] = t.y; B[2] = t.z;
    B[3] = t.y; B[4] = t.w; B[5] = u.x;
    B[6] = t.z; B[7] = u.x; B[8] = u.y;
}

// V_j (1 - q/2)^3 -- the Wendland (dW/dr)/r V_j = cF (1 - q/2)^3 V_j
// without the prefactor cF, which the row sums take once -- and the
// reference separation X_i - X_j of one pair.
template <bool WRAP>
__device__ __forceinline__ float pair_weight(const TlArgs& t, const Wrap& w, const float4& gi, const float4& gj,
                                             float* d) {
    d[0] = gi.x - gj.x;
    d[1] = gi.y - gj.y;
    d[2] = gi.z - gj.z;
    if (WRAP) {
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = wrap1(d[a], w.L[a], w.invL[a]);
    }
    const float r2 = fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2]));
    const float tq = fmaf(t.nhh, __builtin_amdgcn_sqrtf(r2), 1.f);
    return (gj.w * tq) * (tq * tq);
}

// w x into a compensated row sum: step 0 a compensated addition of its own,
// 1 the first and 2 the second of two terms added together (Kahan open and
// close).
__device__ __forceinline__ void accum_step(Kahan& k, float w, float x, int step) {
    if (step == 1) k.open(w, x);
    else if (step == 2) k.close(w, x);
    else accum(k, w, x);
}

// (v_j - v_i) (x) (X_i - X_j) V_j (1 - q/2)^3 into the nine compensated row sums.
template <bool WRAP>
__device__ __forceinline__ void acc_a(const TlArgs& t, const Wrap& w, const float4& gi, const float4& vi,
                                      const float4& gj, const float4& vj, Kahan* L, int step = 0) {
    float d[3];
    const float wt = pair_weight<WRAP>(t, w, gi, gj, d);
    const float dv[3] = {vj.x - vi.x, vj.y - vi.y, vj.z - vi.z};
    const float dw[3] = {wt * d[0], wt * d[1], wt * d[2]};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) accum_step(L[r * 3 + c], dv[r], dw[c], step);
}

// The per-particle end of kernel A (on the group's first lane): dF/dt = L B0,
// then (MODE 0) dF/dt at the caller index or (MODE 1) F += dt dF/dt and the
// position drift on non-fixed rows; A_i = P(F_i) B0_i for kernel B.
template <int MODE>
__device__ __forceinline__ void tl_a_tail(const TlArgs& t, int32_t i, const float* Ld, const float4& vi, bool fixed,
                                          const float4& f0, const float4& f1, float f2,
                                          const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                          const float4* __restrict__ sorted, float4* __restrict__ F0,
                                          float4* __restrict__ F1, float* __restrict__ F2, float4* __restrict__ posS,
                                          float* __restrict__ dFdt, float4* __restrict__ A0, float4* __restrict__ A1,
                                          float* __restrict__ A2) {
    float Fd[9];
    float B[9];
    load_B3(i, geo1, geo2, B);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Fd[r * 3 + c] = Ld[r * 3 + 0] * B[c] + Ld[r * 3 + 1] * B[3 + c] + Ld[r * 3 + 2] * B[6 + c];
    float H[9] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w, f2};
    if (MODE == 0) {
        const int32_t ic = __float_as_int(sorted[i].w);
#pragma unroll
        for (int q = 0; q < 9; ++q) dFdt[(int64_t)ic * 9 + q] = Fd[q];
    } else if (!fixed) {
#pragma unroll
        for (int q = 0; q < 9; ++q) H[q] += t.dt * Fd[q];
        F0[i] = make_float4(H[0], H[1], H[2], H[3]);
        F1[i] = make_float4(H[4], H[5], H[6], H[7]);
        F2[i] = H[8];
        const float4 x = posS[i];
        posS[i] = make_float4(x.x + t.dt * vi.x, x.y + t.dt * vi.y, x.z + t.dt * vi.z, 0.f);
    }
    H[0] -= 1.f;
    H[4] -= 1.f;
    H[8] -= 1.f;
    float P[9];
    pk1_from_H(H, t, P);
    float Ai[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Ai[r * 3 + c] = P[r * 3 + 0] * B[c] + P[r * 3 + 1] * B[3 + c] + P[r * 3 + 2] * B[6 + c];
    A0[i] = make_float4(Ai[0], Ai[1], Ai[2], Ai[3]);
    A1[i] = make_float4(Ai[4], Ai[5], Ai[6], Ai[7]);
    A2[i] = Ai[8];
}

// Kernel A (Eq. 32 and the stress of Eq. 30 / neo-Hookean).  One thread per
// sorted slot; the neighbour records (X_j, V_j and v_j) are gathered one
// entry ahead of the pair being evaluated.  F lives in cell-sorted order
// (F0, F1, F2).  MODE 0: dF/dt -> dFdt at the caller index, F untouched.
// MODE 1: F += dt dF/dt, x += dt v (non-fixed rows).  Both: A_i = P(F_i) B0_i
// (B0 symmetric).
template <int MODE, bool ELL, int LN>
__global__ void __launch_bounds__(BLK) k_tl_a(int32_t n, TlArgs t, Wrap w, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col, int32_t S,
                                              const float4* __restrict__ geo0, const float4* __restrict__ geo1,
                                              const float2* __restrict__ geo2, const float4* __restrict__ sorted,
                                              const float4* __restrict__ VH, float4* __restrict__ F0,
                                              float4* __restrict__ F1, float* __restrict__ F2,
                                              float4* __restrict__ posS, float* __restrict__ dFdt,
                                              float4* __restrict__ A0, float4* __restrict__ A1, float* __restrict__ A2) {
    const int64_t tt = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;
    const int32_t i = (int32_t)(tt / LN);  // sorted slot
    const int sub = (int)(tt % LN);
    if (i >= n) return;
    const float4 gi = ld32(geo0, (uint32_t)i);
    const float4 vi = ld32(VH, (uint32_t)i);
    const bool fixed = vi.w != 0.f;
    const float4 f0 = F0[i], f1 = F1[i];
    const float f2 = F2[i];
    const bool wrap = wave_needs_wrap(w, gi);
    Kahan L[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k].init();
    int64_t k, e, stride;
    row_range<ELL, LN>(i, sub, n, rp, S, k, e, stride);
    int32_t j = k < e ? col[k] : i;
    float4 gj = ld32(geo0, (uint32_t)j), vj = ld32(VH, (uint32_t)j);
    int32_t jn = k + stride < e ? col[k + stride] : i;
    while (k < e) {
        const float4 gn = ld32(geo0, (uint32_t)jn), vn = ld32(VH, (uint32_t)jn);
        jn = k + 2 * stride < e ? col[k + 2 * stride] : i;
        k += stride;
        if (wrap) acc_a<true>(t, w, gi, vi, gj, vj, L);
        else acc_a<false>(t, w, gi, vi, gj, vj, L);
        gj = gn;
        vj = vn;
    }
    float Ld[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Ld[q] = t.cF * group_sum<LN>(L[q]);
    if (sub != 0) return;
    tl_a_tail<MODE>(t, i, Ld, vi, fixed, f0, f1, f2, geo1, geo2, sorted, F0, F1, F2, posS, dFdt, A0, A1, A2);
}

struct ARec {
    float4 g, a0, a1;
    float a2;
};

__device__ __forceinline__ void gather_a(int32_t j, const float4* __restrict__ geo0, const float4* __restrict__ A0,
                                         const float4* __restrict__ A1, const float* __restrict__ A2, ARec& r) {
    const uint32_t u = (uint32_t)j;
    r.g = ld32(geo0, u);
    r.a0 = ld32(A0, u);
    r.a1 = ld32(A1, u);
    r.a2 = ld32(A2, u);
}

// V_j (1 - q/2)^3 (A_i + A_j)(X_i - X_j) into the three compensated row sums.
template <bool WRAP>
__device__ __forceinline__ void acc_b(const TlArgs& t, const Wrap& w, const float4& gi, const float* Ai,
                                      const ARec& b, Kahan* s) {
    float d[3];
    const float wt = pair_weight<WRAP>(t, w, gi, b.g, d);
    accum(s[0], wt, fmaf(Ai[0] + b.a0.x, d[0], fmaf(Ai[1] + b.a0.y, d[1], (Ai[2] + b.a0.z) * d[2])));
    accum(s[1], wt, fmaf(Ai[3] + b.a0.w, d[0], fmaf(Ai[4] + b.a1.x, d[1], (Ai[5] + b.a1.y) * d[2])));
    accum(s[2], wt, fmaf(Ai[6] + b.a1.z, d[0], fmaf(Ai[7] + b.a1.w, d[1], (Ai[8] + b.a2) * d[2])));
}

// Kernel B (Eq. 31), records gathered one entry ahead.  MODE 0: acc (caller
// SoA) = a_i (0 on fixed rows).  MODE 1: ACC[i] = a_i, VH[i] += dt a_i
// (non-fixed rows).
template <int MODE, bool ELL, int LN>
__global__ void __launch_bounds__(BLK) k_tl_b(int32_t n, TlArgs t, Wrap w, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ col, int32_t S,
                                              const float4* __restrict__ geo0, const float4* __restrict__ A0,
                                              const float4* __restrict__ A1, const float* __restrict__ A2,
                                              const float4* __restrict__ sorted, float4* __restrict__ VH,
                                              float4* __restrict__ ACC, float* __restrict__ acc) {
    const int64_t tt = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;
    const int32_t i = (int32_t)(tt / LN);  // sorted slot
    const int sub = (int)(tt % LN);
    if (i >= n) return;
    ARec own;
    gather_a(i, geo0, A0, A1, A2, own);
    const float4 gi = own.g;
    const float Ai[9] = {own.a0.x, own.a0.y, own.a0.z, own.a0.w, own.a1.x, own.a1.y, own.a1.z, own.a1.w, own.a2};
    const float4 vh = VH[i];
    const bool wrap = wave_needs_wrap(w, gi);
    Kahan s[3];
    s[0].init(); s[1].init(); s[2].init();
    int64_t k, e, stride;
    row_range<ELL, LN>(i, sub, n, rp, S, k, e, stride);
    ARec cur, nxt;
    gather_a(k < e ? col[k] : i, geo0, A0, A1, A2, cur);
    int32_t jn = k + stride < e ? col[k + stride] : i;
    while (k < e) {
        gather_a(jn, geo0, A0, A1, A2, nxt);
        jn = k + 2 * stride < e ? col[k + 2 * stride] : i;
        k += stride;
        if (wrap) acc_b<true>(t, w, gi, Ai, cur, s);
        else acc_b<false>(t, w, gi, Ai, cur, s);
        cur = nxt;
    }
    const float fa = t.cF * t.inv_rho0;
    float a[3] = {group_sum<LN>(s[0]) * fa, group_sum<LN>(s[1]) * fa, group_sum<LN>(s[2]) * fa};
    if (sub != 0) return;
    const bool fixed = vh.w != 0.f;
    if (fixed) a[0] = a[1] = a[2] = 0.f;
    if (MODE == 0) {
        const int32_t ic = __float_as_int(sorted[i].w);
        acc[ic] = a[0];
        acc[(int64_t)n + ic] = a[1];
        acc[2 * (int64_t)n + ic] = a[2];
    } else {
        ACC[i] = make_float4(a[0], a[1], a[2], 0.f);
        if (!fixed) VH[i] = make_float4(vh.x + t.dt * a[0], vh.y + t.dt * a[1], vh.z + t.dt * a[2], 0.f);
    }
}

// Kernel B over neighbour windows (fixed-stride rows, four lanes per
// particle): workgroup blk of NT threads takes block blk of P = NT / 4 slots
// and first copies the records of its window (X_j and V_j, A_j) into LDS
// planes; the pairs read them there through 16-bit byte offsets, a lane's
// chunk of M entries in one load.  The rows are padded with the slot itself
// (zero separation: the pair adds nothing).  Same arithmetic as k_tl_b.
template <int HC, int NT>
constexpr int tl_window_waves() {  // waves per SIMD the LDS allows, at most 6 (80 VGPRs)
    constexpr int w = 163840 / (52 * HC) * (NT / 64) / 4;
    return w < 6 ? w : 6;
}

__device__ __forceinline__ void tl_wread(const char* W, uint32_t b, int HC4, ARec& r) {
    r.g = *reinterpret_cast<const float4*>(W + b);
    r.a0 = *reinterpret_cast<const float4*>(W + HC4 + b);
    r.a1 = *reinterpret_cast<const float4*>(W + 2 * HC4 + b);
    r.a2 = *reinterpret_cast<const float*>(W + 3 * HC4 + (b >> 2));
}

// b, made to depend on the pair sum just updated (an empty asm statement
// emits no instruction), so the next record's LDS reads stay after the pair
// that frees its registers.
__device__ __forceinline__ uint32_t tl_after(uint32_t b, const Kahan& k) {
    asm volatile("" : "+v"(b) : "v"(k.s), "v"(k.c));
    return b;
}

// v, required in registers at this point (an empty asm statement that reads
// it: the loads that produce it are complete here, and none of them is moved
// into a guarded block after it).
__device__ __forceinline__ void tl_held(const float4& v) {
    asm volatile("" : : "v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}
__device__ __forceinline__ void tl_held(float v) { asm volatile("" : : "v"(v)); }

// The lane's chunks of window entries of one row (records from LDS, two in
// flight), in the order k_tl_b takes them.  (Its three sums take each pair
// on its own: two at a time made this kernel slower, 92.6 against 83.9 us
// per launch on the 1.6M plate.)
template <bool WRAP, int M>
__device__ __forceinline__ void tl_row_w(const TlArgs& t, const Wrap& w, const char* W, int HC4,
                                         const uint16_t* __restrict__ colw, uint32_t at0, uint32_t cs, int32_t nchunk,
                                         const float4& gi, const float* Ai, Kahan* s) {
    for (int32_t c = 0; c < nchunk; ++c) {
        uint32_t e[M / 2];
        load_chunk<M>(colw, at0 + (uint32_t)c * cs, e);
        ARec A, B;
        tl_wread(W, e[0] & 0xffffu, HC4, A);
        tl_wread(W, e[0] >> 16, HC4, B);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < M; q += 2) {
            acc_b<WRAP>(t, w, gi, Ai, A, s);
            if (q + 2 < M) tl_wread(W, tl_after(e[q / 2 + 1] & 0xffffu, s[0]), HC4, A);
            __builtin_amdgcn_sched_barrier(0);
            acc_b<WRAP>(t, w, gi, Ai, B, s);
            if (q + 3 < M) tl_wread(W, tl_after(e[q / 2 + 1] >> 16, s[0]), HC4, B);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int MODE, int M, int HC, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tl_window_waves<HC, NT>())))
k_tl_bw(int32_t n, TlArgs t, Wrap w, const uint16_t* __restrict__ colw, int32_t Sp,
        const int32_t* __restrict__ woff, const int32_t* __restrict__ wlist, const float4* __restrict__ geo0,
        const float4* __restrict__ A0, const float4* __restrict__ A1, const float* __restrict__ A2,
        const float4* __restrict__ sorted, float4* __restrict__ VH, float4* __restrict__ ACC,
        float* __restrict__ acc) {
    constexpr int L = 4;
    constexpr int HC4 = 16 * HC;  // bytes of a float4 plane
    __shared__ __attribute__((aligned(16))) char W[3 * HC4 + 4 * HC];
    const int32_t blk = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int32_t w0 = woff[blk], wn = woff[blk + 1] - w0;
    {
        // a thread per record, at most KC records each: the slot indices
        // are loaded first, then the records, then written to LDS, so the
        // copy waits on two memory latencies, not 2 KC.  Threads past the
        // window's end load its last record again (every window holds the
        // block's own slots, so it is never empty) and write nothing.
        constexpr int KC = (HC + NT - 1) / NT;
        uint32_t j[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) j[r] = (uint32_t)wlist[w0 + min((int32_t)threadIdx.x + r * NT, wn - 1)];
        float4 g[KC], a0[KC], a1[KC];
        float a2[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            g[r] = ld32(geo0, j[r]);
            a0[r] = ld32(A0, j[r]);
            a1[r] = ld32(A1, j[r]);
            a2[r] = ld32(A2, j[r]);
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            tl_held(g[r]);
            tl_held(a0[r]);
            tl_held(a1[r]);
            tl_held(a2[r]);
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            const int32_t k = (int32_t)threadIdx.x + r * NT;
            if (k < wn) {
                *reinterpret_cast<float4*>(W + 16 * k) = g[r];
                *reinterpret_cast<float4*>(W + HC4 + 16 * k) = a0[r];
                *reinterpret_cast<float4*>(W + 2 * HC4 + 16 * k) = a1[r];
                *reinterpret_cast<float*>(W + 3 * HC4 + 4 * k) = a2[r];
            }
        }
    }
    const int sub = (int)(threadIdx.x % L);
    const int32_t ig = blk * (NT / L) + (int32_t)(threadIdx.x / L);
    const bool valid = ig < n;
    const int32_t i = valid ? ig : n - 1;
    const uint32_t self = 16u * (uint32_t)(i - blk * (NT / L));
    const uint32_t at0 = ((uint32_t)i * L + (uint32_t)sub) * (uint32_t)(M / 2);
    const uint32_t cs = (uint32_t)n * L * (uint32_t)(M / 2);
    const int32_t nchunk = Sp / (L * M);
    const float4 vh = VH[i];
    __syncthreads();
    ARec own;
    tl_wread(W, self, HC4, own);
    const float4 gi = own.g;
    const float Ai[9] = {own.a0.x, own.a0.y, own.a0.z, own.a0.w, own.a1.x, own.a1.y, own.a1.z, own.a1.w, own.a2};
    const bool wrap = wave_needs_wrap(w, gi);
    Kahan s[3];
    s[0].init(); s[1].init(); s[2].init();
    if (wrap) tl_row_w<true, M>(t, w, W, HC4, colw, at0, cs, nchunk, gi, Ai, s);
    else tl_row_w<false, M>(t, w, W, HC4, colw, at0, cs, nchunk, gi, Ai, s);
    const float fa = t.cF * t.inv_rho0;
    float a[3] = {group_sum<L>(s[0]) * fa, group_sum<L>(s[1]) * fa, group_sum<L>(s[2]) * fa};
    if (sub != 0 || !valid) return;
    const bool fixed = vh.w != 0.f;
    if (fixed) a[0] = a[1] = a[2] = 0.f;
    if (MODE == 0) {
        const int32_t ic = __float_as_int(sorted[i].w);
        acc[ic] = a[0];
        acc[(int64_t)n + ic] = a[1];
        acc[2 * (int64_t)n + ic] = a[2];
    } else {
        ACC[i] = make_float4(a[0], a[1], a[2], 0.f);
        if (!fixed) VH[i] = make_float4(vh.x + t.dt * a[0], vh.y + t.dt * a[1], vh.z + t.dt * a[2], 0.f);
    }
}

// Kernel A over the same neighbour windows: the window's reference records
// (X_j, V_j) and half-step velocities (v_j, fixed flag) copied into two LDS
// planes, the pairs read there and enter the nine compensated sums two at a
// time; the per-particle end as in k_tl_a.
template <int HC, int NT>
constexpr int tl_window_waves_a() {  // waves per SIMD the LDS allows, at most 6 (80 VGPRs)
    constexpr int w = 163840 / (32 * HC) * (NT / 64) / 4;
    return w < 6 ? w : 6;
}

template <bool WRAP, int M>
__device__ __forceinline__ void tl_row_aw(const TlArgs& t, const Wrap& w, const char* W, int HC4,
                                          const uint16_t* __restrict__ colw, uint32_t at0, uint32_t cs,
                                          int32_t nchunk, const float4& gi, const float4& vi, Kahan* L) {
    for (int32_t c = 0; c < nchunk; ++c) {
        uint32_t e[M / 2];
        load_chunk<M>(colw, at0 + (uint32_t)c * cs, e);
        float4 ga = *reinterpret_cast<const float4*>(W + (e[0] & 0xffffu));
        float4 va = *reinterpret_cast<const float4*>(W + HC4 + (e[0] & 0xffffu));
        float4 gb = *reinterpret_cast<const float4*>(W + (e[0] >> 16));
        float4 vb = *reinterpret_cast<const float4*>(W + HC4 + (e[0] >> 16));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < M; q += 2) {
            acc_a<WRAP>(t, w, gi, vi, ga, va, L, 1);
            if (q + 2 < M) {
                const uint32_t b = tl_after(e[q / 2 + 1] & 0xffffu, L[0]);
                ga = *reinterpret_cast<const float4*>(W + b);
                va = *reinterpret_cast<const float4*>(W + HC4 + b);
            }
            __builtin_amdgcn_sched_barrier(0);
            acc_a<WRAP>(t, w, gi, vi, gb, vb, L, 2);
            if (q + 3 < M) {
                const uint32_t b = tl_after(e[q / 2 + 1] >> 16, L[0]);
                gb = *reinterpret_cast<const float4*>(W + b);
                vb = *reinterpret_cast<const float4*>(W + HC4 + b);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int MODE, int M, int HC, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tl_window_waves_a<HC, NT>())))
k_tl_aw(int32_t n, TlArgs t, Wrap w, const uint16_t* __restrict__ colw, int32_t Sp, const int32_t* __restrict__ woff,
        const int32_t* __restrict__ wlist, const float4* __restrict__ geo0, const float4* __restrict__ geo1,
        const float2* __restrict__ geo2, const float4* __restrict__ sorted, const float4* __restrict__ VH,
        float4* __restrict__ F0, float4* __restrict__ F1, float* __restrict__ F2, float4* __restrict__ posS,
        float* __restrict__ dFdt, float4* __restrict__ A0, float4* __restrict__ A1, float* __restrict__ A2) {
    constexpr int L = 4;
    constexpr int HC4 = 16 * HC;
    __shared__ __attribute__((aligned(16))) char W[2 * HC4];
    const int32_t blk = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int32_t w0 = woff[blk], wn = woff[blk + 1] - w0;
    {
        // the window copy in three phases (slot indices, records, LDS
        // writes), as in k_tl_bw
        constexpr int KC = (HC + NT - 1) / NT;
        uint32_t j[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) j[r] = (uint32_t)wlist[w0 + min((int32_t)threadIdx.x + r * NT, wn - 1)];
        float4 g[KC], v[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            g[r] = ld32(geo0, j[r]);
            v[r] = ld32(VH, j[r]);
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            tl_held(g[r]);
            tl_held(v[r]);
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            const int32_t k = (int32_t)threadIdx.x + r * NT;
            if (k < wn) {
                *reinterpret_cast<float4*>(W + 16 * k) = g[r];
                *reinterpret_cast<float4*>(W + HC4 + 16 * k) = v[r];
            }
        }
    }
    const int sub = (int)(threadIdx.x % L);
    const int32_t ig = blk * (NT / L) + (int32_t)(threadIdx.x / L);
    const bool valid = ig < n;
    const int32_t i = valid ? ig : n - 1;
    const uint32_t self = 16u * (uint32_t)(i - blk * (NT / L));
    const uint32_t at0 = ((uint32_t)i * L + (uint32_t)sub) * (uint32_t)(M / 2);
    const uint32_t cs = (uint32_t)n * L * (uint32_t)(M / 2);
    const int32_t nchunk = Sp / (L * M);
    const float4 f0 = F0[i], f1 = F1[i];
    const float f2 = F2[i];
    __syncthreads();
    const float4 gi = *reinterpret_cast<const float4*>(W + self);
    const float4 vi = *reinterpret_cast<const float4*>(W + HC4 + self);
    const bool fixed = vi.w != 0.f;
    const bool wrap = wave_needs_wrap(w, gi);
    Kahan Ls[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ls[k].init();
    if (wrap) tl_row_aw<true, M>(t, w, W, HC4, colw, at0, cs, nchunk, gi, vi, Ls);
    else tl_row_aw<false, M>(t, w, W, HC4, colw, at0, cs, nchunk, gi, vi, Ls);
    float Ld[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Ld[q] = t.cF * group_sum<L>(Ls[q]);
    if (sub != 0 || !valid) return;
    tl_a_tail<MODE>(t, i, Ld, vi, fixed, f0, f1, f2, geo1, geo2, sorted, F0, F1, F2, posS, dFdt, A0, A1, A2);
}

// F (caller [n][9]) and positions (caller SoA, optional) into sorted order, and back.
__global__ void k_tl_pack(int32_t n, const float4* __restrict__ sorted, const float* __restrict__ F,
                          const float* __restrict__ pos, float4* __restrict__ F0, float4* __restrict__ F1,
                          float* __restrict__ F2, float4* __restrict__ posS) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = __float_as_int(sorted[s].w);
    const float* f = F + (int64_t)i * 9;
    F0[s] = make_float4(f[0], f[1], f[2], f[3]);
    F1[s] = make_float4(f[4], f[5], f[6], f[7]);
    F2[s] = f[8];
    if (pos) posS[s] = make_float4(pos[i], pos[(int64_t)n + i], pos[2 * (int64_t)n + i], 0.f);
}

__global__ void k_tl_unpack(int32_t n, const float4* __restrict__ sorted, const float4* __restrict__ F0,
                            const float4* __restrict__ F1, const float* __restrict__ F2,
                            const float4* __restrict__ posS, float* __restrict__ F, float* __restrict__ pos) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = __float_as_int(sorted[s].w);
    const float4 a = F0[s], b = F1[s];
    float* f = F + (int64_t)i * 9;
    f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
    f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
    f[8] = F2[s];
    const float4 x = posS[s];
    pos[i] = x.x;
    pos[(int64_t)n + i] = x.y;
    pos[2 * (int64_t)n + i] = x.z;
}

// VH = v + half_dt * a (0 and flagged on fixed rows); ACC = a
__global__ void k_tl_init(int32_t n, float half_dt, const float4* __restrict__ sorted, const float* __restrict__ vel,
                          const float* __restrict__ acc, const int32_t* __restrict__ fixed, float4* __restrict__ VH,
                          float4* __restrict__ ACC) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t i = __float_as_int(sorted[s].w);
    bool fx = fixed && fixed[i] != 0;
    float4 a = acc ? make_float4(acc[i], acc[(int64_t)n + i], acc[2 * (int64_t)n + i], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    if (fx) a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ACC) ACC[s] = a;
    VH[s] = fx ? make_float4(0.f, 0.f, 0.f, 1.f)
               : make_float4(vel[i] + half_dt * a.x, vel[(int64_t)n + i] + half_dt * a.y,
                             vel[2 * (int64_t)n + i] + half_dt * a.z, 0.f);
}

// v = VH - half_dt ACC; acc = ACC
__global__ void k_tl_finish(int32_t n, float half_dt, const float4* __restrict__ sorted,
                            const float4* __restrict__ VH, const float4* __restrict__ ACC, float* __restrict__ vel,
                            float* __restrict__ acc) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t i = __float_as_int(sorted[s].w);
    float4 v = VH[s], a = ACC[s];
    bool fx = v.w != 0.f;
    vel[i] = fx ? 0.f : v.x - half_dt * a.x;
    vel[(int64_t)n + i] = fx ? 0.f : v.y - half_dt * a.y;
    vel[2 * (int64_t)n + i] = fx ? 0.f : v.z - half_dt * a.z;
    acc[i] = a.x;
    acc[(int64_t)n + i] = a.y;
    acc[2 * (int64_t)n + i] = a.z;
}

TlArgs make_args(const sph_ctx* c, const sph_tlsph_params* p) {
    TlArgs t{};
    t.lam = (float)(p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu)));
    t.G = (float)(p->E / (2.0 * (1.0 + p->nu)));
    t.inv_rho0 = (float)(1.0 / p->rho0);
    t.dt = (float)p->dt;
    t.half_dt = (float)(0.5 * p->dt);
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, 3, c->dom.h);
    t.hinv = kc.hinv;
    t.cF = kc.cF;
    t.nhh = -0.5f * kc.hinv;
    t.model = p->model;
    return t;
}

int check(sph_ctx* c, const sph_tlsph_params* p, const char* who) {
    if (!c) return SPH_ERR_ARG;
    if (c->dim != 3) return sph_fail(c, SPH_ERR_ARG, "%s: 3-D only", who);
    if (!c->bound || !c->geo_valid)
        return sph_fail(c, SPH_ERR_STATE, "%s: needs a bound configuration and a cached correction", who);
    if (c->dom.kernel != SPH_WENDLAND) return sph_fail(c, SPH_ERR_ARG, "%s: Wendland kernel only", who);
    if (!p) return sph_fail(c, SPH_ERR_ARG, "%s: params NULL", who);
    if (!(p->rho0 > 0.0) || !(p->E > 0.0) || !(p->nu > -1.0 && p->nu < 0.5))
        return sph_fail(c, SPH_ERR_ARG, "%s: need rho0 > 0, E > 0, -1 < nu < 0.5", who);
    if (p->model != 0 && p->model != 1) return sph_fail(c, SPH_ERR_ARG, "%s: model must be 0 or 1", who);
    return SPH_OK;
}

// Lanes per particle of the total-Lagrangian pair loops: the most (up to
// 4) that leave each lane at least three row entries (measured on the
// cantilever plate, rows of 26 and 56 entries).  Tuning override
// SPH_TLSPH_LANES = 1, 2 or 4.
int tl_lanes(const sph_ctx* c) {
    if (const char* e = getenv("SPH_TLSPH_LANES")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4) return v;
    }
    const double avg = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    int L = 1;
    while (L < 4 && avg / (2 * L) >= 3.0) L <<= 1;
    return L;
}

int ensure_scratch(sph_ctx* c) {
    size_t n = (size_t)(c->n > 0 ? c->n : 1);
    SPH_HIP(c, c->ua.ensure(n * sizeof(float4)));   // VH
    SPH_HIP(c, c->ub.ensure(n * sizeof(float4)));   // ACC
    SPH_HIP(c, c->ta.ensure(n * sizeof(float4)));   // A0
    SPH_HIP(c, c->tb.ensure(n * sizeof(float4)));   // A1
    SPH_HIP(c, c->tc.ensure(n * sizeof(float)));    // A2
    SPH_HIP(c, c->fa.ensure(n * sizeof(float4)));   // F0
    SPH_HIP(c, c->fb.ensure(n * sizeof(float4)));   // F1
    SPH_HIP(c, c->fc.ensure(n * sizeof(float)));    // F2
    SPH_HIP(c, c->pa.ensure(n * sizeof(float4)));   // current positions
    int r = sph_ell_prepare(c);
    if (r) return r;
    // kernel B reads its neighbour records from LDS windows (four lanes per
    // particle, blocks of 128 slots); tuning override SPH_TLSPH_WINDOW=0
    const char* e = getenv("SPH_TLSPH_WINDOW");
    if (tl_lanes(c) != 4 || (e && strcmp(e, "0") == 0)) {
        c->wtl.state = -1;
        c->wtl.P = 0;
        return SPH_OK;
    }
    return sph_windows_prepare(c, c->wtl, 4, 128);
}

template <int MODE, int M, int HC>
void launch_aw_h(sph_ctx* c, const TlArgs& t, const Wrap& w, float* dFdt) {
    const NeighbourWindows& wd = c->wtl;
    constexpr int NT = 512;
    hipLaunchKernelGGL((k_tl_aw<MODE, M, HC, NT>), dim3(grid_for(c->n, NT / 4)), dim3(NT), 0, c->stream, c->n, t, w,
                       wd.col.as<uint16_t>(), wd.Sp, wd.off.as<int32_t>(), wd.list.as<int32_t>(), c->geo0.as<float4>(),
                       c->geo1.as<float4>(), c->geo2.as<float2>(), c->sorted.as<float4>(), c->ua.as<float4>(),
                       c->fa.as<float4>(), c->fb.as<float4>(), c->fc.as<float>(), c->pa.as<float4>(), dFdt,
                       c->ta.as<float4>(), c->tb.as<float4>(), c->tc.as<float>());
}

template <int MODE, int M>
void launch_aw_m(sph_ctx* c, const TlArgs& t, const Wrap& w, float* dFdt) {
    const int32_t mx = c->wtl.max;
    if (mx <= 512) launch_aw_h<MODE, M, 512>(c, t, w, dFdt);
    else if (mx <= 768) launch_aw_h<MODE, M, 768>(c, t, w, dFdt);
    else launch_aw_h<MODE, M, 1024>(c, t, w, dFdt);
}

template <int MODE>
void launch_a(sph_ctx* c, const TlArgs& t, const Wrap& w, float* dFdt) {
    const int LN = tl_lanes(c);
    if (LN == 4 && c->wtl.state == 1) {
        const int M = c->wtl.M;
        if (M == 12) launch_aw_m<MODE, 12>(c, t, w, dFdt);
        else if (M == 10) launch_aw_m<MODE, 10>(c, t, w, dFdt);
        else if (M == 8) launch_aw_m<MODE, 8>(c, t, w, dFdt);
        else launch_aw_m<MODE, 6>(c, t, w, dFdt);
        return;
    }
    dim3 g(grid_for((int64_t)c->n * LN, BLK)), bl(BLK);
    const bool ell = c->ell_state == 1;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g, bl, 0, c->stream, c->n, t, w, ell ? nullptr : c->rp_s.as<int64_t>(),
                           ell ? c->colE.as<int32_t>() : c->col_s.as<int32_t>(), ell ? c->ell_S : 0,
                           c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), c->sorted.as<float4>(),
                           c->ua.as<float4>(), c->fa.as<float4>(), c->fb.as<float4>(), c->fc.as<float>(),
                           c->pa.as<float4>(), dFdt, c->ta.as<float4>(), c->tb.as<float4>(), c->tc.as<float>());
    };
    if (ell) {
        if (LN == 1) go(k_tl_a<MODE, true, 1>);
        else if (LN == 2) go(k_tl_a<MODE, true, 2>);
        else go(k_tl_a<MODE, true, 4>);
    } else {
        if (LN == 1) go(k_tl_a<MODE, false, 1>);
        else if (LN == 2) go(k_tl_a<MODE, false, 2>);
        else go(k_tl_a<MODE, false, 4>);
    }
}

template <int MODE, int M, int HC>
void launch_bw_h(sph_ctx* c, const TlArgs& t, const Wrap& w, float* acc) {
    const NeighbourWindows& wd = c->wtl;
    constexpr int NT = 512;
    hipLaunchKernelGGL((k_tl_bw<MODE, M, HC, NT>), dim3(grid_for(c->n, NT / 4)), dim3(NT), 0, c->stream, c->n, t, w,
                       wd.col.as<uint16_t>(), wd.Sp, wd.off.as<int32_t>(), wd.list.as<int32_t>(), c->geo0.as<float4>(),
                       c->ta.as<float4>(), c->tb.as<float4>(), c->tc.as<float>(), c->sorted.as<float4>(),
                       c->ua.as<float4>(), c->ub.as<float4>(), acc);
}

template <int MODE, int M>
void launch_bw_m(sph_ctx* c, const TlArgs& t, const Wrap& w, float* acc) {
    const int32_t mx = c->wtl.max;
    if (mx <= 512) launch_bw_h<MODE, M, 512>(c, t, w, acc);
    else if (mx <= 768) launch_bw_h<MODE, M, 768>(c, t, w, acc);
    else launch_bw_h<MODE, M, 1024>(c, t, w, acc);
}

template <int MODE>
void launch_b(sph_ctx* c, const TlArgs& t, const Wrap& w, float* acc) {
    const int LN = tl_lanes(c);
    c->tlsph_path = SPH_PATH_GENERIC;
    if (LN == 4 && c->wtl.state == 1) {
        c->tlsph_path = SPH_PATH_WINDOWS;
        const int M = c->wtl.M;
        if (M == 12) launch_bw_m<MODE, 12>(c, t, w, acc);
        else if (M == 10) launch_bw_m<MODE, 10>(c, t, w, acc);
        else if (M == 8) launch_bw_m<MODE, 8>(c, t, w, acc);
        else launch_bw_m<MODE, 6>(c, t, w, acc);
        return;
    }
    dim3 g(grid_for((int64_t)c->n * LN, BLK)), bl(BLK);
    const bool ell = c->ell_state == 1;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, g, bl, 0, c->stream, c->n, t, w, ell ? nullptr : c->rp_s.as<int64_t>(),
                           ell ? c->colE.as<int32_t>() : c->col_s.as<int32_t>(), ell ? c->ell_S : 0,
                           c->geo0.as<float4>(), c->ta.as<float4>(), c->tb.as<float4>(), c->tc.as<float>(),
                           c->sorted.as<float4>(), c->ua.as<float4>(), c->ub.as<float4>(), acc);
    };
    if (ell) {
        if (LN == 1) go(k_tl_b<MODE, true, 1>);
        else if (LN == 2) go(k_tl_b<MODE, true, 2>);
        else go(k_tl_b<MODE, true, 4>);
    } else {
        if (LN == 1) go(k_tl_b<MODE, false, 1>);
        else if (LN == 2) go(k_tl_b<MODE, false, 2>);
        else go(k_tl_b<MODE, false, 4>);
    }
}

}  // namespace

extern "C" {

int sph_tlsph_rhs(sph_ctx* c, const sph_tlsph_params* p, const float* vel, const float* F, const int32_t* fixed,
                  float* dF_dt, float* acc) {
    int r = check(c, p, "sph_tlsph_rhs");
    if (r) return r;
    if (c->n == 0) return SPH_OK;
    if (!vel || !F || !dF_dt || !acc) return sph_fail(c, SPH_ERR_ARG, "sph_tlsph_rhs: NULL array");
    r = ensure_scratch(c);
    if (r) return r;
    TlArgs t = make_args(c, p);
    Wrap w = make_wrap(c);
    dim3 g(grid_for(c->n, BLK)), bl(BLK);
    const float4* sorted = c->sorted.as<float4>();
    hipLaunchKernelGGL(k_tl_init, g, bl, 0, c->stream, c->n, 0.f, sorted, vel, (const float*)nullptr, fixed,
                       c->ua.as<float4>(), (float4*)nullptr);
    hipLaunchKernelGGL(k_tl_pack, g, bl, 0, c->stream, c->n, sorted, F, (const float*)nullptr, c->fa.as<float4>(),
                       c->fb.as<float4>(), c->fc.as<float>(), c->pa.as<float4>());
    launch_a<0>(c, t, w, dF_dt);
    launch_b<0>(c, t, w, acc);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_tlsph_step(sph_ctx* c, const sph_tlsph_params* p, const int32_t* fixed, float* pos, float* vel, float* F,
                   float* acc, int32_t nsteps) {
    int r = check(c, p, "sph_tlsph_step");
    if (r) return r;
    if (nsteps < 0) return sph_fail(c, SPH_ERR_ARG, "sph_tlsph_step: nsteps < 0");
    if (!(p->dt > 0.0)) return sph_fail(c, SPH_ERR_ARG, "sph_tlsph_step: dt must be > 0");
    if (c->n == 0 || nsteps == 0) return SPH_OK;
    if (!pos || !vel || !F || !acc) return sph_fail(c, SPH_ERR_ARG, "sph_tlsph_step: NULL array");
    r = ensure_scratch(c);
    if (r) return r;
    TlArgs t = make_args(c, p);
    Wrap w = make_wrap(c);
    dim3 g(grid_for(c->n, BLK)), bl(BLK);
    const float4* sorted = c->sorted.as<float4>();
    hipLaunchKernelGGL(k_tl_init, g, bl, 0, c->stream, c->n, t.half_dt, sorted, vel, acc, fixed, c->ua.as<float4>(),
                       c->ub.as<float4>());
    hipLaunchKernelGGL(k_tl_pack, g, bl, 0, c->stream, c->n, sorted, F, pos, c->fa.as<float4>(), c->fb.as<float4>(),
                       c->fc.as<float>(), c->pa.as<float4>());
    for (int32_t s = 0; s < nsteps; ++s) {
        launch_a<1>(c, t, w, nullptr);
        launch_b<1>(c, t, w, nullptr);
    }
    hipLaunchKernelGGL(k_tl_finish, g, bl, 0, c->stream, c->n, t.half_dt, sorted, c->ua.as<float4>(),
                       c->ub.as<float4>(), vel, acc);
    hipLaunchKernelGGL(k_tl_unpack, g, bl, 0, c->stream, c->n, sorted, c->fa.as<float4>(), c->fb.as<float4>(),
                       c->fc.as<float>(), c->pa.as<float4>(), F, pos);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
