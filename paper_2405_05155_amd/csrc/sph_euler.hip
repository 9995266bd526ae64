// sph_euler.hip -- Riemann-based Eulerian SPH (Eq. 19, mass and momentum
// rows) with the corrected gradient (Eq. 28) and the limited linearised
// Riemann solver (Eqs. 26-27), and its Heun time stepping.
//
// State layout: one float4 record per particle (drho, m_x, m_y, m_z), so a
// neighbour's whole state is one 16-byte gather; geometry comes from the
// context's cached records (position, V, B upper triangle).
#include "sph_internal.h"

namespace {

constexpr int BLK = 256;

struct EulerArgs {
    float c, c2, cinv, c2inv;
    float rho0;    // EOS reference density
    float rho_ref; // rho = rho_ref + drho
    float poff;    // rho_ref - rho0 (so p = c^2 (drho + poff))
    float eta, mu2; // limiter coefficient; 2 mu
    float dt;
    float hinv, cF; // Wendland (dW/dr)/r = cF (1 - q/2)^3
};

template <int DIM>
__global__ void k_pack_state(int32_t n, const float* __restrict__ drho, const float* __restrict__ mom,
                             float4* __restrict__ U) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    U[i] = make_float4(drho[i], mom[i], mom[(int64_t)n + i], DIM == 3 ? mom[2 * (int64_t)n + i] : 0.f);
}

template <int DIM>
__global__ void k_unpack_state(int32_t n, const float4* __restrict__ U, float* __restrict__ drho,
                               float* __restrict__ mom) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 u = U[i];
    drho[i] = u.x;
    mom[i] = u.y;
    mom[(int64_t)n + i] = u.z;
    if (DIM == 3) mom[2 * (int64_t)n + i] = u.w;
}

// STAGE 0: write rates; 1: Uout = U + dt R(U); 2: Uout = (U0 + U + dt R(U)) / 2
// (Uout may alias U0: each thread reads and writes only its own record).
template <int DIM, int STAGE>
__global__ void __launch_bounds__(BLK) k_euler(int32_t n, BoxArgs b, EulerArgs ea, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, const float4* __restrict__ geo0,
                                               const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                               const float4* __restrict__ U, const float4* U0, float4* Uout,
                                               float* __restrict__ drho_dt, float* __restrict__ dmom_dt) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 gi = geo0[i];
    float Bi[6];
    if (DIM == 2) {
        float2 t = reinterpret_cast<const float2*>(geo1)[i];
        Bi[0] = gi.w; Bi[1] = t.x; Bi[2] = t.y;
    } else {
        float4 t = geo1[i];
        float2 u = geo2[i];
        Bi[0] = t.x; Bi[1] = t.y; Bi[2] = t.z; Bi[3] = t.w; Bi[4] = u.x; Bi[5] = u.y;
    }
    float4 ui = U[i];
    float rhoi = ea.rho_ref + ui.x;
    float invi = fast_rcp(rhoi);
    float vi[3] = {ui.y * invi, ui.z * invi, DIM == 3 ? ui.w * invi : 0.f};
    float pi_ = ea.c2 * (ui.x + ea.poff);

    Kahan sr, sm[DIM];
    sr.init();
#pragma unroll
    for (int a = 0; a < DIM; ++a) sm[a].init();

    int64_t e = row_ptr[i + 1];
    for (int64_t k = row_ptr[i]; k < e; ++k) {
        int32_t j = col[k];
        float4 gj = geo0[j];
        float Bj[6];
        if (DIM == 2) {
            float2 t = reinterpret_cast<const float2*>(geo1)[j];
            Bj[0] = gj.w; Bj[1] = t.x; Bj[2] = t.y;
        } else {
            float4 t = geo1[j];
            float2 u = geo2[j];
            Bj[0] = t.x; Bj[1] = t.y; Bj[2] = t.z; Bj[3] = t.w; Bj[4] = u.x; Bj[5] = u.y;
        }
        float4 uj = U[j];
        float d[3];
        d[0] = min_image(gi.x - gj.x, b.L[0], b.halfL[0], b.periodic[0]);
        d[1] = min_image(gi.y - gj.y, b.L[1], b.halfL[1], b.periodic[1]);
        d[2] = DIM == 3 ? min_image(gi.z - gj.z, b.L[2], b.halfL[2], b.periodic[2]) : 0.f;
        float r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 == 0.f) continue;
        float rinv = rsqrtf(r2);
        float q = r2 * rinv * ea.hinv;
        float F = wendland_F(q, ea.cF);  // (dW/dr)/r
        float Vj = DIM == 2 ? gj.z : gj.w;
        // grad W = F d;  corrected: gc = (B_i + B_j)/2 grad W
        float g[3] = {F * d[0], F * d[1], F * d[2]};
        float gc[3];
        if (DIM == 2) {
            gc[0] = 0.5f * ((Bi[0] + Bj[0]) * g[0] + (Bi[1] + Bj[1]) * g[1]);
            gc[1] = 0.5f * ((Bi[1] + Bj[1]) * g[0] + (Bi[2] + Bj[2]) * g[1]);
            gc[2] = 0.f;
        } else {
            gc[0] = 0.5f * ((Bi[0] + Bj[0]) * g[0] + (Bi[1] + Bj[1]) * g[1] + (Bi[2] + Bj[2]) * g[2]);
            gc[1] = 0.5f * ((Bi[1] + Bj[1]) * g[0] + (Bi[3] + Bj[3]) * g[1] + (Bi[4] + Bj[4]) * g[2]);
            gc[2] = 0.5f * ((Bi[2] + Bj[2]) * g[0] + (Bi[4] + Bj[4]) * g[1] + (Bi[5] + Bj[5]) * g[2]);
        }
        // Riemann problem along n = (r_j - r_i)/r, left = i, right = j
        float nrm[3] = {-d[0] * rinv, -d[1] * rinv, -d[2] * rinv};
        float rhoj = ea.rho_ref + uj.x;
        float invj = fast_rcp(rhoj);
        float vj[3] = {uj.y * invj, uj.z * invj, DIM == 3 ? uj.w * invj : 0.f};
        float pj = ea.c2 * (uj.x + ea.poff);
        float ul = vi[0] * nrm[0] + vi[1] * nrm[1] + vi[2] * nrm[2];
        float ur = vj[0] * nrm[0] + vj[1] * nrm[1] + vj[2] * nrm[2];
        float rhobar = 0.5f * (rhoi + rhoj);
        float beta = fminf(ea.eta * fmaxf((ul - ur) * ea.cinv, 0.f), 1.f);
        float umean = 0.5f * (ul + ur);
        float ustar = umean + 0.5f * beta * beta * (pi_ - pj) * fast_rcp(rhobar * ea.c);
        float pstar = 0.5f * (pi_ + pj) + 0.5f * beta * rhobar * ea.c * (ul - ur);
        float du = ustar - umean;
        float vs[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) vs[a] = 0.5f * (vi[a] + vj[a]) + du * nrm[a];
        float rhostar = ea.rho0 + pstar * ea.c2inv;
        float vg = vs[0] * gc[0] + vs[1] * gc[1] + vs[2] * gc[2];
        float m2V = -2.f * Vj;
        sr.add(m2V * rhostar * vg);
        float visc = ea.mu2 * Vj * F;
#pragma unroll
        for (int a = 0; a < DIM; ++a) sm[a].add(m2V * (rhostar * vs[a] * vg + pstar * gc[a]) + visc * (vi[a] - vj[a]));
    }
    float R[4] = {sr.value(), sm[0].value(), sm[1].value(), DIM == 3 ? sm[DIM - 1].value() : 0.f};
    if (STAGE == 0) {
        drho_dt[i] = R[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) dmom_dt[(int64_t)a * n + i] = R[1 + a];
    } else if (STAGE == 1) {
        Uout[i] = make_float4(ui.x + ea.dt * R[0], ui.y + ea.dt * R[1], ui.z + ea.dt * R[2],
                              DIM == 3 ? ui.w + ea.dt * R[3] : 0.f);
    } else {
        float4 u0 = U0[i];
        Uout[i] = make_float4(0.5f * (u0.x + (ui.x + ea.dt * R[0])), 0.5f * (u0.y + (ui.y + ea.dt * R[1])),
                              0.5f * (u0.z + (ui.z + ea.dt * R[2])),
                              DIM == 3 ? 0.5f * (u0.w + (ui.w + ea.dt * R[3])) : 0.f);
    }
}

EulerArgs make_args(const sph_ctx* c, const sph_euler_params* p) {
    EulerArgs a{};
    a.c = (float)p->c;
    a.c2 = (float)(p->c * p->c);
    a.cinv = (float)(1.0 / p->c);
    a.c2inv = (float)(1.0 / (p->c * p->c));
    a.rho0 = (float)p->rho0;
    a.rho_ref = (float)p->rho_ref;
    a.poff = (float)(p->rho_ref - p->rho0);
    a.eta = (float)p->eta;
    a.mu2 = (float)(2.0 * p->mu);
    a.dt = (float)p->dt;
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, c->dim, c->dom.h);
    a.hinv = kc.hinv;
    a.cF = kc.cF;
    return a;
}

int check(sph_ctx* c, const sph_euler_params* p, const char* who) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound || !c->geo_valid)
        return sph_fail(c, SPH_ERR_STATE, "%s: needs a bound configuration and a cached correction", who);
    if (c->dom.kernel != SPH_WENDLAND) return sph_fail(c, SPH_ERR_ARG, "%s: Wendland kernel only", who);
    if (!p) return sph_fail(c, SPH_ERR_ARG, "%s: params NULL", who);
    if (!(p->c > 0.0)) return sph_fail(c, SPH_ERR_ARG, "%s: sound speed must be > 0", who);
    if (!(p->eta >= 0.0) || !(p->mu >= 0.0)) return sph_fail(c, SPH_ERR_ARG, "%s: eta and mu must be >= 0", who);
    return SPH_OK;
}

template <int STAGE>
void launch(sph_ctx* c, const EulerArgs& ea, const float4* U, const float4* U0, float4* Uout, float* dr, float* dm) {
    if (c->dim == 2)
        hipLaunchKernelGGL((k_euler<2, STAGE>), dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, c->box, ea,
                           c->row_ptr.as<int64_t>(), c->col.as<int32_t>(), c->geo0.as<float4>(), c->geo1.as<float4>(),
                           c->geo2.as<float2>(), U, U0, Uout, dr, dm);
    else
        hipLaunchKernelGGL((k_euler<3, STAGE>), dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, c->box, ea,
                           c->row_ptr.as<int64_t>(), c->col.as<int32_t>(), c->geo0.as<float4>(), c->geo1.as<float4>(),
                           c->geo2.as<float2>(), U, U0, Uout, dr, dm);
}

int pack(sph_ctx* c, const float* drho, const float* mom, float4* U) {
    if (c->dim == 2)
        hipLaunchKernelGGL(k_pack_state<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, drho, mom, U);
    else
        hipLaunchKernelGGL(k_pack_state<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, drho, mom, U);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // namespace

extern "C" {

int sph_euler_rhs(sph_ctx* c, const sph_euler_params* p, const float* drho, const float* mom, float* drho_dt,
                  float* dmom_dt) {
    int r = check(c, p, "sph_euler_rhs");
    if (r) return r;
    if (c->n == 0) return SPH_OK;
    if (!drho || !mom || !drho_dt || !dmom_dt) return sph_fail(c, SPH_ERR_ARG, "sph_euler_rhs: NULL array");
    SPH_HIP(c, c->ua.ensure((size_t)c->n * sizeof(float4)));
    r = pack(c, drho, mom, c->ua.as<float4>());
    if (r) return r;
    EulerArgs ea = make_args(c, p);
    launch<0>(c, ea, c->ua.as<float4>(), nullptr, nullptr, drho_dt, dmom_dt);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

int sph_euler_step(sph_ctx* c, const sph_euler_params* p, float* drho, float* mom, int32_t nsteps) {
    int r = check(c, p, "sph_euler_step");
    if (r) return r;
    if (nsteps < 0) return sph_fail(c, SPH_ERR_ARG, "sph_euler_step: nsteps < 0");
    if (!(p->dt > 0.0)) return sph_fail(c, SPH_ERR_ARG, "sph_euler_step: dt must be > 0");
    if (c->n == 0 || nsteps == 0) return SPH_OK;
    if (!drho || !mom) return sph_fail(c, SPH_ERR_ARG, "sph_euler_step: NULL array");
    SPH_HIP(c, c->ua.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->ub.ensure((size_t)c->n * sizeof(float4)));
    float4* U = c->ua.as<float4>();
    float4* Us = c->ub.as<float4>();
    r = pack(c, drho, mom, U);
    if (r) return r;
    EulerArgs ea = make_args(c, p);
    for (int32_t s = 0; s < nsteps; ++s) {
        launch<1>(c, ea, U, nullptr, Us, nullptr, nullptr);
        launch<2>(c, ea, Us, U, U, nullptr, nullptr);
    }
    SPH_LAUNCH_CHECK(c);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_unpack_state<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, U, drho, mom);
    else
        hipLaunchKernelGGL(k_unpack_state<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, U, drho, mom);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
