// sph_euler.hip -- Riemann-based Eulerian SPH (Eq. 19, mass and momentum
// rows) with the corrected gradient (Eq. 28) and the limited linearised
// Riemann solver (Eqs. 26-27), and its Heun time stepping.
//
// State layout: one float4 record per particle (drho, m_x, m_y, m_z), so a
// neighbour's whole state is one 16-byte gather; geometry comes from the
// context's cached records (position, V, B upper triangle).  All records
// live in cell-sorted (Morton) order; the caller's arrays are gathered in
// and scattered out at the caller index.
#include "sph_internal.h"

#include <cstdlib>

namespace {

constexpr int BLK = 256;

struct EulerArgs {
    float c, c2, c2inv;
    float rho0;     // EOS reference density
    float rho_ref;  // rho = rho_ref + drho
    float poff;     // rho_ref - rho0 (so p = c^2 (drho + poff))
    float eta_c;    // limiter coefficient / c
    float mu4;      // 4 mu (multiplies (dW/dr)/r / 2)
    float dt;
    float hinv, cFh; // Wendland (dW/dr)/r / 2 = cFh (1 - q/2)^3
    float L[3], invL[3];  // periodic lengths (invL = 0 on open axes)
};

// Conserved record U = (drho, m_x, m_y, m_z) and primitive record
// P = (drho, v_x, v_y, v_z) per particle.  Neighbours are read through P
// (one 16-byte gather gives density deviation and velocity), so the pair
// loop needs no division; each stage writes both records of its result.
template <int DIM>
__device__ __forceinline__ float4 primitive(const float4& u, float rho_ref) {
    float rho = rho_ref + u.x;
    return make_float4(u.x, u.y / rho, u.z / rho, DIM == 3 ? u.w / rho : 0.f);
}

template <int DIM>
__global__ void k_pack_state(int32_t n, float rho_ref, const float4* __restrict__ sorted,
                             const float* __restrict__ drho, const float* __restrict__ mom, float4* __restrict__ U,
                             float4* __restrict__ P) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t i = __float_as_int(sorted[s].w);
    float4 u = make_float4(drho[i], mom[i], mom[(int64_t)n + i], DIM == 3 ? mom[2 * (int64_t)n + i] : 0.f);
    U[s] = u;
    P[s] = primitive<DIM>(u, rho_ref);
}

template <int DIM>
__global__ void k_unpack_state(int32_t n, const float4* __restrict__ sorted, const float4* __restrict__ U,
                               float* __restrict__ drho, float* __restrict__ mom) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t i = __float_as_int(sorted[s].w);
    float4 u = U[s];
    drho[i] = u.x;
    mom[i] = u.y;
    mom[(int64_t)n + i] = u.z;
    if (DIM == 3) mom[2 * (int64_t)n + i] = u.w;
}

// Periodic wrap without branches: d - L rint(d / L) (invL = 0 on open axes).
// For |d| < L the correction is 0 or +-L and, for coordinates that are
// multiples of a power of two, exact.
__device__ __forceinline__ float wrap(float d, float L, float invL) { return fmaf(-L, rintf(d * invL), d); }

// STAGE 0: write rates; 1: Uout = U + dt R(U); 2: Uout = (U0 + U + dt R(U)) / 2.
// Stage 1 and 2 also write Pout, the primitive record of Uout.
// Uout / Pout may alias U0 / the own records of the stage input: each
// particle's records are read and written only by its own lane group, and
// neighbours are gathered from P, which a stage never writes in place.
// L lanes per particle: lane `sub` of the group takes the neighbours
// row_ptr[i] + sub, + sub + L, ...; the compensated partial sums are combined
// by group_sum and lane 0 of the group writes the result.
template <int DIM, int STAGE, int L>
__global__ void __launch_bounds__(BLK) k_euler(int32_t n, EulerArgs ea, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, const float4* __restrict__ geo0,
                                               const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                               const float4* U, const float4* __restrict__ P, const float4* U0,
                                               float4* Uout, float4* Pout, const float4* __restrict__ sorted,
                                               float* __restrict__ drho_dt, float* __restrict__ dmom_dt) {
    // i below is the cell-sorted slot; XCD-contiguous block order
    int64_t t = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * blockDim.x + threadIdx.x;
    int32_t i = (int32_t)(t / L);
    const int sub = (int)(t % L);
    // whole groups leave together (n * L is not always a multiple of the block)
    if (i >= n) return;
    constexpr int NBU = DIM == 2 ? 3 : 6;  // upper-triangle entries of B
    float4 gi = geo0[i];
    float xi[3] = {gi.x, gi.y, gi.z};
    float Bi[NBU];
    if (DIM == 2) {
        float2 t2 = reinterpret_cast<const float2*>(geo1)[i];
        Bi[0] = gi.w; Bi[1] = t2.x; Bi[2] = t2.y;
    } else {
        float4 t4 = geo1[i];
        float2 u2 = geo2[i];
        Bi[0] = t4.x; Bi[1] = t4.y; Bi[2] = t4.z; Bi[3] = t4.w; Bi[4] = u2.x; Bi[5] = u2.y;
    }
    float4 pi4 = P[i];
    float rhoi = ea.rho_ref + pi4.x;
    float vi[3] = {pi4.y, pi4.z, pi4.w};
    float pi_ = ea.c2 * (pi4.x + ea.poff);

    Kahan sr, sm[DIM];
    sr.init();
#pragma unroll
    for (int a = 0; a < DIM; ++a) sm[a].init();

    // The next column index is loaded one iteration ahead; the pair is
    // branch-free (coincident particles get zero weight), so all gathers of
    // an iteration are issued before its arithmetic.
    int64_t e = row_ptr[i + 1];
    int64_t k = row_ptr[i] + sub;
    int32_t jn = k < e ? col[k] : i;
    while (k < e) {
        int32_t j = jn;
        k += L;
        jn = k < e ? col[k] : i;
        float4 gj = geo0[j];
        float Bs[NBU];
        if (DIM == 2) {
            float2 t2 = reinterpret_cast<const float2*>(geo1)[j];
            Bs[0] = Bi[0] + gj.w; Bs[1] = Bi[1] + t2.x; Bs[2] = Bi[2] + t2.y;
        } else {
            float4 t4 = geo1[j];
            float2 u2 = geo2[j];
            Bs[0] = Bi[0] + t4.x; Bs[1] = Bi[1] + t4.y; Bs[2] = Bi[2] + t4.z;
            Bs[3] = Bi[3] + t4.w; Bs[4] = Bi[4] + u2.x; Bs[5] = Bi[5] + u2.y;
        }
        float4 pj4 = P[j];
        float xj[3] = {gj.x, gj.y, gj.z};
        float d[DIM];
        float r2 = 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            d[a] = wrap(xi[a] - xj[a], ea.L[a], ea.invL[a]);
            r2 = fmaf(d[a], d[a], r2);
        }
        const bool live = r2 > 0.f;
        float rinv = live ? __builtin_amdgcn_rsqf(r2) : 0.f;
        float tq = fmaf(-0.5f * ea.hinv, r2 * rinv, 1.f);  // 1 - q/2
        float Fh = ea.cFh * tq * tq * tq;                   // (dW/dr)/r / 2
        float Vj = live ? (DIM == 2 ? gj.z : gj.w) : 0.f;
        // gc = (B_i + B_j)/2 grad W = Fh (B_i + B_j) d
        float gc[DIM];
        if (DIM == 2) {
            gc[0] = Fh * fmaf(Bs[0], d[0], Bs[1] * d[1]);
            gc[1] = Fh * fmaf(Bs[1], d[0], Bs[2] * d[1]);
        } else {
            gc[0] = Fh * fmaf(Bs[0], d[0], fmaf(Bs[1], d[1], Bs[2] * d[2]));
            gc[1] = Fh * fmaf(Bs[1], d[0], fmaf(Bs[3], d[1], Bs[4] * d[2]));
            gc[2] = Fh * fmaf(Bs[2], d[0], fmaf(Bs[4], d[1], Bs[5] * d[2]));
        }
        // Riemann problem along n = -d / r (from i to j), left = i, right = j
        float vj[3] = {pj4.y, pj4.z, pj4.w};
        float dvd = 0.f, svd = 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            dvd = fmaf(vi[a] - vj[a], d[a], dvd);
            svd = fmaf(vi[a] + vj[a], d[a], svd);
        }
        float du_lr = -dvd * rinv;               // u_l - u_r
        float umean = -0.5f * svd * rinv;        // (u_l + u_r) / 2
        float rhoj = ea.rho_ref + pj4.x;
        float pj = ea.c2 * (pj4.x + ea.poff);
        float rhobar_c = 0.5f * ea.c * (rhoi + rhoj);
        float beta = fminf(ea.eta_c * fmaxf(du_lr, 0.f), 1.f);
        float hb = 0.5f * beta;
        float du = hb * beta * (pi_ - pj) * fast_rcp(rhobar_c);   // u* - mean
        float pstar = fmaf(0.5f, pi_ + pj, hb * rhobar_c * du_lr);
        float rhostar = fmaf(pstar, ea.c2inv, ea.rho0);
        // v* = (v_i + v_j)/2 + (u* - mean) n
        float dun = -du * rinv;
        float vs[DIM];
        float vg = 0.f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            vs[a] = fmaf(0.5f, vi[a] + vj[a], dun * d[a]);
            vg = fmaf(vs[a], gc[a], vg);
        }
        float m2V = -2.f * Vj;
        float rvg = rhostar * vg;
        sr.add(m2V * rvg);
        float visc = ea.mu4 * Vj * Fh;  // 2 mu V (dW/dr)/r
#pragma unroll
        for (int a = 0; a < DIM; ++a) sm[a].add(fmaf(m2V, fmaf(rvg, vs[a], pstar * gc[a]), visc * (vi[a] - vj[a])));
    }
    float R[4];
    R[0] = group_sum<L>(sr);
#pragma unroll
    for (int a = 0; a < DIM; ++a) R[1 + a] = group_sum<L>(sm[a]);
    if (DIM == 2) R[3] = 0.f;
    if (sub != 0) return;
    if (STAGE == 0) {
        int32_t ic = __float_as_int(sorted[i].w);
        drho_dt[ic] = R[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) dmom_dt[(int64_t)a * n + ic] = R[1 + a];
        return;
    }
    float4 ui = U[i];
    float4 un;
    if (STAGE == 1) {
        un = make_float4(ui.x + ea.dt * R[0], ui.y + ea.dt * R[1], ui.z + ea.dt * R[2],
                         DIM == 3 ? ui.w + ea.dt * R[3] : 0.f);
    } else {
        float4 u0 = U0[i];
        un = make_float4(0.5f * (u0.x + (ui.x + ea.dt * R[0])), 0.5f * (u0.y + (ui.y + ea.dt * R[1])),
                         0.5f * (u0.z + (ui.z + ea.dt * R[2])),
                         DIM == 3 ? 0.5f * (u0.w + (ui.w + ea.dt * R[3])) : 0.f);
    }
    Uout[i] = un;
    Pout[i] = primitive<DIM>(un, ea.rho_ref);
}

EulerArgs make_args(const sph_ctx* c, const sph_euler_params* p) {
    EulerArgs a{};
    a.c = (float)p->c;
    a.c2 = (float)(p->c * p->c);
    a.c2inv = (float)(1.0 / (p->c * p->c));
    a.rho0 = (float)p->rho0;
    a.rho_ref = (float)p->rho_ref;
    a.poff = (float)(p->rho_ref - p->rho0);
    a.eta_c = (float)(p->eta / p->c);
    a.mu4 = (float)(4.0 * p->mu);
    a.dt = (float)p->dt;
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, c->dim, c->dom.h);
    a.hinv = kc.hinv;
    a.cFh = 0.5f * kc.cF;
    for (int ax = 0; ax < 3; ++ax) {
        a.L[ax] = c->box.L[ax];
        a.invL[ax] = c->box.periodic[ax] ? (float)(1.0 / c->box.Ld[ax]) : 0.f;
    }
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

struct StageIO {
    const float4* U;
    const float4* P;
    const float4* U0;
    float4* Uout;
    float4* Pout;
    float* dr;
    float* dm;
};

template <int DIM, int STAGE, int L>
void launch_l(sph_ctx* c, const EulerArgs& ea, const StageIO& io) {
    hipLaunchKernelGGL((k_euler<DIM, STAGE, L>), dim3(grid_for((int64_t)c->n * L, BLK)), dim3(BLK), 0, c->stream, c->n,
                       ea, c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), c->geo0.as<float4>(), c->geo1.as<float4>(),
                       c->geo2.as<float2>(), io.U, io.P, io.U0, io.Uout, io.Pout, c->sorted.as<float4>(), io.dr, io.dm);
}

// Lanes per particle: enough lane groups to give every SIMD several waves
// (the chip holds 256 CUs x 4 SIMDs), and a few neighbours per lane.
int lanes_per_particle(const sph_ctx* c) {
    // tuning override: SPH_EULER_LANES = 1, 2, 4 or 8
    static int forced = [] {
        const char* e = getenv("SPH_EULER_LANES");
        int v = e ? atoi(e) : 0;
        return (v == 1 || v == 2 || v == 4 || v == 8) ? v : 0;
    }();
    if (forced) return forced;
    const int64_t target = 256LL * 4 * 16 * 64;  // two rounds of 8 waves per SIMD
    double avg = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    int L = 1;
    while (L < 8 && (int64_t)c->n * L < target && avg / (2 * L) >= 2.0) L <<= 1;
    return L;
}

template <int STAGE>
void launch(sph_ctx* c, const EulerArgs& ea, const StageIO& io) {
    int L = lanes_per_particle(c);
    if (c->dim == 2) {
        if (L == 1) launch_l<2, STAGE, 1>(c, ea, io);
        else if (L == 2) launch_l<2, STAGE, 2>(c, ea, io);
        else if (L == 4) launch_l<2, STAGE, 4>(c, ea, io);
        else launch_l<2, STAGE, 8>(c, ea, io);
    } else {
        if (L == 1) launch_l<3, STAGE, 1>(c, ea, io);
        else if (L == 2) launch_l<3, STAGE, 2>(c, ea, io);
        else if (L == 4) launch_l<3, STAGE, 4>(c, ea, io);
        else launch_l<3, STAGE, 8>(c, ea, io);
    }
}

int pack(sph_ctx* c, float rho_ref, const float* drho, const float* mom, float4* U, float4* P) {
    if (c->dim == 2)
        hipLaunchKernelGGL(k_pack_state<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, rho_ref,
                           c->sorted.as<float4>(), drho, mom, U, P);
    else
        hipLaunchKernelGGL(k_pack_state<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, rho_ref,
                           c->sorted.as<float4>(), drho, mom, U, P);
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
    SPH_HIP(c, c->ta.ensure((size_t)c->n * sizeof(float4)));
    EulerArgs ea = make_args(c, p);
    r = pack(c, ea.rho_ref, drho, mom, c->ua.as<float4>(), c->ta.as<float4>());
    if (r) return r;
    StageIO io{c->ua.as<float4>(), c->ta.as<float4>(), nullptr, nullptr, nullptr, drho_dt, dmom_dt};
    launch<0>(c, ea, io);
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
    SPH_HIP(c, c->ta.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->tb.ensure((size_t)c->n * sizeof(float4)));
    float4* U = c->ua.as<float4>();
    float4* Us = c->ub.as<float4>();
    float4* P = c->ta.as<float4>();
    float4* Ps = c->tb.as<float4>();
    EulerArgs ea = make_args(c, p);
    r = pack(c, ea.rho_ref, drho, mom, U, P);
    if (r) return r;
    // stage 1 gathers P, writes (U*, P*); stage 2 gathers P*, writes (U, P) in place
    StageIO s1{U, P, nullptr, Us, Ps, nullptr, nullptr};
    StageIO s2{Us, Ps, U, U, P, nullptr, nullptr};
    for (int32_t s = 0; s < nsteps; ++s) {
        launch<1>(c, ea, s1);
        launch<2>(c, ea, s2);
    }
    SPH_LAUNCH_CHECK(c);
    if (c->dim == 2)
        hipLaunchKernelGGL(k_unpack_state<2>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                           c->sorted.as<float4>(), U, drho, mom);
    else
        hipLaunchKernelGGL(k_unpack_state<3>, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                           c->sorted.as<float4>(), U, drho, mom);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
