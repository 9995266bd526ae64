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
// resolution (no I - C^{-1} or ln J cancellation).  Velocity, acceleration
// and A records live in cell-sorted (Morton) order; F and positions stay in
// the caller's arrays and are accessed at the caller index of each slot.
#include "sph_internal.h"

namespace {

constexpr int BLK = 256;

struct TlArgs {
    float lam, G, inv_rho0, dt, half_dt;
    float hinv, cF;
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
    float4 t = geo1[i];
    float2 u = geo2[i];
    B[0] = t.x; B[1] = t.y; B[2] = t.z;
    B[3] = t.y; B[4] = t.w; B[5] = u.x;
    B[6] = t.z; B[7] = u.x; B[8] = u.y;
}

// Kernel A.  MODE 0: dF/dt -> dFdt (caller), F untouched.  MODE 1: F += dt dF/dt,
// x += dt v (non-fixed rows).  Both: A_i = P(F_i) B0_i (B0 symmetric).
template <int MODE>
__global__ void __launch_bounds__(BLK) k_tl_a(int32_t n, BoxArgs b, TlArgs t, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const float4* __restrict__ geo0,
                                              const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                              const float4* __restrict__ sorted, const float4* __restrict__ VH,
                                              float* __restrict__ F, float* __restrict__ dFdt, float* __restrict__ pos,
                                              float4* __restrict__ A0, float4* __restrict__ A1, float* __restrict__ A2) {
    int32_t i = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;  // sorted slot
    if (i >= n) return;
    const int32_t ic = __float_as_int(sorted[i].w);                                     // caller index
    float4 gi = geo0[i];
    float4 vi = VH[i];
    bool fixed = vi.w != 0.f;
    Kahan L[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) L[k].init();
    int64_t e = row_ptr[i + 1];
    for (int64_t k = row_ptr[i]; k < e; ++k) {
        int32_t j = col[k];
        float4 gj = geo0[j];
        float4 vj = VH[j];
        float d0 = min_image(gi.x - gj.x, b.L[0], b.halfL[0], b.periodic[0]);
        float d1 = min_image(gi.y - gj.y, b.L[1], b.halfL[1], b.periodic[1]);
        float d2 = min_image(gi.z - gj.z, b.L[2], b.halfL[2], b.periodic[2]);
        float r2 = d0 * d0 + d1 * d1 + d2 * d2;
        float q = sqrtf(r2) * t.hinv;
        float w = wendland_F(q, t.cF) * gj.w;  // V_j (dW/dr)/r
        float dv[3] = {(vj.x - vi.x) * w, (vj.y - vi.y) * w, (vj.z - vi.z) * w};
        float d[3] = {d0, d1, d2};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) L[r * 3 + c].add(dv[r] * d[c]);
    }
    float B[9];
    load_B3(i, geo1, geo2, B);
    float Ld[9], Fd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ld[k] = L[k].value();
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Fd[r * 3 + c] = Ld[r * 3 + 0] * B[c] + Ld[r * 3 + 1] * B[3 + c] + Ld[r * 3 + 2] * B[6 + c];
    float* Fi = F + (int64_t)ic * 9;
    float H[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) H[k] = Fi[k];
    if (MODE == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) dFdt[(int64_t)ic * 9 + k] = Fd[k];
    } else if (!fixed) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            H[k] += t.dt * Fd[k];
            Fi[k] = H[k];
        }
        pos[ic] += t.dt * vi.x;
        pos[(int64_t)n + ic] += t.dt * vi.y;
        pos[2 * (int64_t)n + ic] += t.dt * vi.z;
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

// Kernel B.  MODE 0: acc (caller SoA) = a_i (0 on fixed rows).
// MODE 1: ACC[i] = a_i, VH[i] += dt a_i (non-fixed rows).
template <int MODE>
__global__ void __launch_bounds__(BLK) k_tl_b(int32_t n, BoxArgs b, TlArgs t, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const float4* __restrict__ geo0,
                                              const float4* __restrict__ A0, const float4* __restrict__ A1,
                                              const float* __restrict__ A2, const float4* __restrict__ sorted,
                                              float4* __restrict__ VH, float4* __restrict__ ACC,
                                              float* __restrict__ acc) {
    int32_t i = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;  // sorted slot
    if (i >= n) return;
    float4 gi = geo0[i];
    float4 a0 = A0[i], a1 = A1[i];
    float Ai[9] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, A2[i]};
    Kahan s[3];
    s[0].init(); s[1].init(); s[2].init();
    int64_t e = row_ptr[i + 1];
    for (int64_t k = row_ptr[i]; k < e; ++k) {
        int32_t j = col[k];
        float4 gj = geo0[j];
        float4 b0 = A0[j], b1 = A1[j];
        float b2 = A2[j];
        float d0 = min_image(gi.x - gj.x, b.L[0], b.halfL[0], b.periodic[0]);
        float d1 = min_image(gi.y - gj.y, b.L[1], b.halfL[1], b.periodic[1]);
        float d2 = min_image(gi.z - gj.z, b.L[2], b.halfL[2], b.periodic[2]);
        float r2 = d0 * d0 + d1 * d1 + d2 * d2;
        float q = sqrtf(r2) * t.hinv;
        float w = wendland_F(q, t.cF) * gj.w;
        float g0 = w * d0, g1 = w * d1, g2 = w * d2;
        s[0].add((Ai[0] + b0.x) * g0 + (Ai[1] + b0.y) * g1 + (Ai[2] + b0.z) * g2);
        s[1].add((Ai[3] + b0.w) * g0 + (Ai[4] + b1.x) * g1 + (Ai[5] + b1.y) * g2);
        s[2].add((Ai[6] + b1.z) * g0 + (Ai[7] + b1.w) * g1 + (Ai[8] + b2) * g2);
    }
    float a[3] = {s[0].value() * t.inv_rho0, s[1].value() * t.inv_rho0, s[2].value() * t.inv_rho0};
    float4 vh = VH[i];
    bool fixed = vh.w != 0.f;
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

int ensure_scratch(sph_ctx* c) {
    size_t n = (size_t)(c->n > 0 ? c->n : 1);
    SPH_HIP(c, c->ua.ensure(n * sizeof(float4)));   // VH
    SPH_HIP(c, c->ub.ensure(n * sizeof(float4)));   // ACC
    SPH_HIP(c, c->ta.ensure(n * sizeof(float4)));   // A0
    SPH_HIP(c, c->tb.ensure(n * sizeof(float4)));   // A1
    SPH_HIP(c, c->tc.ensure(n * sizeof(float)));    // A2
    return SPH_OK;
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
    dim3 g(grid_for(c->n, BLK)), bl(BLK);
    const float4* sorted = c->sorted.as<float4>();
    hipLaunchKernelGGL(k_tl_init, g, bl, 0, c->stream, c->n, 0.f, sorted, vel, (const float*)nullptr, fixed,
                       c->ua.as<float4>(), (float4*)nullptr);
    // F is only read in MODE 0
    hipLaunchKernelGGL(k_tl_a<0>, g, bl, 0, c->stream, c->n, c->box, t, c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(),
                       c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), sorted, c->ua.as<float4>(),
                       const_cast<float*>(F), dF_dt, (float*)nullptr, c->ta.as<float4>(), c->tb.as<float4>(),
                       c->tc.as<float>());
    hipLaunchKernelGGL(k_tl_b<0>, g, bl, 0, c->stream, c->n, c->box, t, c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(),
                       c->geo0.as<float4>(), c->ta.as<float4>(), c->tb.as<float4>(), c->tc.as<float>(), sorted,
                       c->ua.as<float4>(), (float4*)nullptr, acc);
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
    dim3 g(grid_for(c->n, BLK)), bl(BLK);
    const float4* sorted = c->sorted.as<float4>();
    hipLaunchKernelGGL(k_tl_init, g, bl, 0, c->stream, c->n, t.half_dt, sorted, vel, acc, fixed, c->ua.as<float4>(),
                       c->ub.as<float4>());
    for (int32_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL(k_tl_a<1>, g, bl, 0, c->stream, c->n, c->box, t, c->rp_s.as<int64_t>(),
                           c->col_s.as<int32_t>(), c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(),
                           sorted, c->ua.as<float4>(), F, (float*)nullptr, pos, c->ta.as<float4>(), c->tb.as<float4>(),
                           c->tc.as<float>());
        hipLaunchKernelGGL(k_tl_b<1>, g, bl, 0, c->stream, c->n, c->box, t, c->rp_s.as<int64_t>(),
                           c->col_s.as<int32_t>(), c->geo0.as<float4>(), c->ta.as<float4>(), c->tb.as<float4>(),
                           c->tc.as<float>(), sorted, c->ua.as<float4>(), c->ub.as<float4>(), (float*)nullptr);
    }
    hipLaunchKernelGGL(k_tl_finish, g, bl, 0, c->stream, c->n, t.half_dt, sorted, c->ua.as<float4>(),
                       c->ub.as<float4>(), vel, acc);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
