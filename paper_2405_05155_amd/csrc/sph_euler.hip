// sph_euler.hip -- Riemann-based Eulerian SPH (Eq. 19) with the corrected
// gradient (Eq. 28) and its Heun time stepping: the weakly compressible
// mass and momentum rows with the limited linearised Riemann solver
// (Eqs. 26-27), and (2-D) the compressible rows with the energy equation and
// the HLLC solver (Eqs. 20-22) with its limiter (Eqs. 24-25), one stage
// kernel for both.
//
// State layout: one float4 conserved record per particle ((drho, m) or, for
// the compressible rows, (rho, m_x, m_y, E)) and one float4 primitive record
// ((drho, v) or (rho, v_x, v_y, p)), so a neighbour's whole state is one
// 16-byte gather; geometry comes from the context's cached records
// (position, V, B upper triangle).  All records live in cell-sorted (Morton)
// order; the caller's arrays are gathered in and scattered out at the caller
// index.
#include "sph_internal.h"

#include <cstdlib>
#include <cstring>

namespace {

constexpr int BLK = 256;

struct EulerArgs {
    float c, c2, c2inv;
    float hc;       // c / 2
    float rho0;     // EOS reference density
    float rho_ref;  // rho = rho_ref + drho
    float poff;     // rho_ref - rho0 (so p = c^2 (drho + poff))
    float eta_c;    // limiter coefficient / c
    float mu_tr;    // 2 mu / d (multiplies tr(B_i + B_j) V_j (dW/dr)/r / 2)
    float dt;
    float hinv, cFh; // Wendland (dW/dr)/r / 2 = cFh (1 - q/2)^3
    // per-particle kernel, which evaluates each pair with the factors that
    // do not depend on the partner taken out of the row sums:
    float nhh;              // -hinv / 2
    float c2x2, c2x2poff;   // 2 c^2, 2 c^2 poff (2 p = 2 c^2 drho + 2 c^2 poff)
    float nec;              // -eta / c
    float qc2inv;           // 1 / (4 c^2)
    float kmu;              // -4 mu / d
    float fr, fm;           // row factors of the continuity and momentum sums: -cFh, -cFh / 2
    float inv2c, crho0x2;   // 1 / (2 c), 2 c rho0 (3-D records: c rho_j = 2 p_j / (2 c) + c rho0)
    // compressible rows (limited HLLC, ideal gas; 2-D)
    float gamma, ig1, gm1;  // gamma, 1 / (gamma - 1), gamma - 1
    float eta_h;            // limiter coefficient
    float fh;               // row factor of the compressible sums: -cF
    float L[3], invL[3];  // periodic lengths (invL = 0 on open axes)
    float lo[3];          // box corner
    float margin;         // a particle this far from every periodic face needs no wrap
};

// Conserved record U = (drho, m_x, m_y, m_z) and primitive record
// P = (drho, v_x, v_y, v_z) per particle.  Neighbours are read through P
// (one 16-byte gather gives density deviation and velocity), so the pair
// loop needs no division; each stage writes both records of its result.
template <int DIM>
__device__ __forceinline__ float4 primitive(const float4& u, float rho_ref) {
    const float inv = fast_rcp(rho_ref + u.x);
    return make_float4(u.x, u.y * inv, u.z * inv, DIM == 3 ? u.w * inv : 0.f);
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

// Gathered records of one neighbour: geometry (2-D (x, y, V, B00) and
// (B01, B11); 3-D (x, y, z, V), (B00, B01, B02, B11) and (B12, B22)) and the
// primitive state (drho, v).
template <int DIM>
struct NbrRec {
    float4 g0, g1, pr;
    float2 g2;
};

template <int DIM>
__device__ __forceinline__ void gather_nbr(int32_t j, const float4* __restrict__ geo0,
                                           const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                           const float4* __restrict__ P, NbrRec<DIM>& r) {
    const uint32_t u = (uint32_t)j;
    r.g0 = ld32(geo0, u);
    if (DIM == 2) {
        const float2 t = ld32(reinterpret_cast<const float2*>(geo1), u);
        r.g1 = make_float4(t.x, t.y, 0.f, 0.f);
        r.g2 = make_float2(0.f, 0.f);
    } else {
        r.g1 = ld32(geo1, u);
        r.g2 = ld32(geo2, u);
    }
    r.pr = ld32(P, u);
}

// Own particle's quantities for its pair loop.
template <int DIM>
struct OwnState {
    float x[3];
    float B[DIM == 2 ? 3 : 6];  // upper triangle of B
    float v[3];
    float p2;    // 2 p_i
    float crho;  // c (rho_i + rho_ref): c (rho_i + rho_j) = crho + c drho_j
    // compressible rows: density, pressure, sound speed, impedance, total energy
    float rho, p, c, z, Et;
};

// One pair (i, j) of Eq. (19) with the corrected gradient (Eq. 28) and the
// limited Riemann solution (Eqs. 26-27).  The factors that do not depend on
// the partner are applied to the compensated row sums afterwards: with
// w = V_j (1 - q/2)^3, G = (B_i + B_j) d, d = x_i - x_j and the kernel's
// (dW/dr)/r = cF (1 - q/2)^3,
//   drho/dt  = -cF/2 sum_j w rho* (2 v* . G),
//   dm/dt    = -cF/4 sum_j w [ rho* (2 v* . G) (2 v*) + 4 p* G
//                             - 4 mu / d tr(B_i + B_j) (v_i - v_j) ],
// the same terms as -2 V_j (rho* v* v* + p* I) (B_i + B_j)/2 grad W plus the
// viscous pair term.  The Riemann problem is solved in doubled variables
// (2 p, c (rho_i + rho_j), 2 (u* - mean), 4 p*) so that each step is one
// fused multiply-add.  Branch-free: a coincident partner (r = 0, also the
// particle itself standing in for a padding entry) gets zero weight.
template <int DIM, bool WRAP>
__device__ __forceinline__ void accumulate_pair(const EulerArgs& ea, const OwnState<DIM>& o, const NbrRec<DIM>& nb,
                                                Kahan& sr, Kahan* sm) {
    constexpr int NBU = DIM == 2 ? 3 : 6;
    const float4 gj = nb.g0;
    float Bs[NBU];
    if (DIM == 2) {
        Bs[0] = o.B[0] + gj.w; Bs[1] = o.B[1] + nb.g1.x; Bs[2] = o.B[2] + nb.g1.y;
    } else {
        Bs[0] = o.B[0] + nb.g1.x; Bs[1] = o.B[1] + nb.g1.y; Bs[2] = o.B[2] + nb.g1.z;
        Bs[3] = o.B[3] + nb.g1.w; Bs[4] = o.B[4] + nb.g2.x; Bs[5] = o.B[5] + nb.g2.y;
    }
    const float4 pj4 = nb.pr;
    const float xj[3] = {gj.x, gj.y, gj.z};
    const float vj[3] = {pj4.y, pj4.z, pj4.w};
    float d[DIM], dv[DIM];
    float r2 = 0.f, dvd = 0.f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        d[a] = o.x[a] - xj[a];
        if (WRAP) d[a] = wrap(d[a], ea.L[a], ea.invL[a]);
        r2 = fmaf(d[a], d[a], r2);
        dv[a] = o.v[a] - vj[a];
        dvd = fmaf(dv[a], d[a], dvd);
    }
    const bool live = r2 > 0.f;
    const float rinv = live ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float tq = fmaf(ea.nhh, r2 * rinv, 1.f);  // 1 - q/2
    const float Vj = live ? (DIM == 2 ? gj.z : gj.w) : 0.f;
    const float w = (Vj * tq) * (tq * tq);
    float G[DIM];
    if (DIM == 2) {
        G[0] = fmaf(Bs[0], d[0], Bs[1] * d[1]);
        G[1] = fmaf(Bs[1], d[0], Bs[2] * d[1]);
    } else {
        G[0] = fmaf(Bs[0], d[0], fmaf(Bs[1], d[1], Bs[2] * d[2]));
        G[1] = fmaf(Bs[1], d[0], fmaf(Bs[3], d[1], Bs[4] * d[2]));
        G[2] = fmaf(Bs[2], d[0], fmaf(Bs[4], d[1], Bs[5] * d[2]));
    }
    // Riemann problem along n = -d / r (from i to j), left = i, right = j:
    // a = u_r - u_l, beta = min(eta max(u_l - u_r, 0) / c, 1)
    const float a = dvd * rinv;
    const float beta = __builtin_amdgcn_fmed3f(ea.nec * a, 0.f, 1.f);
    const float pj2 = fmaf(ea.c2x2, pj4.x, ea.c2x2poff);
    const float crho = fmaf(ea.c, pj4.x, o.crho);
    const float du2 = ((beta * beta) * (o.p2 - pj2)) * fast_rcp(crho);
    const float p4 = fmaf(-(beta * crho), a, o.p2 + pj2);
    const float rhostar = fmaf(p4, ea.qc2inv, ea.rho0);
    // 2 v* = v_i + v_j + 2 (u* - mean) n
    const float dn = du2 * rinv;
    float vs2[DIM];
    float vg2 = 0.f;
#pragma unroll
    for (int a2 = 0; a2 < DIM; ++a2) {
        vs2[a2] = fmaf(-dn, d[a2], o.v[a2] + vj[a2]);
        vg2 = fmaf(vs2[a2], G[a2], vg2);
    }
    const float rh = rhostar * vg2;
    accum(sr, w, rh);
    const float trB = DIM == 2 ? Bs[0] + Bs[2] : (Bs[0] + Bs[3]) + Bs[5];
    const float kv = ea.kmu * trB;
#pragma unroll
    for (int a2 = 0; a2 < DIM; ++a2) accum(sm[a2], w, fmaf(rh, vs2[a2], fmaf(p4, G[a2], kv * dv[a2])));
}

// One pair (i, j) of the compressible system (Eq. 19, all three rows; 2-D)
// with the corrected gradient (Eq. 28) and the limited HLLC interface state
// (Eqs. 20-22, limited by Eqs. 24-25), Riemann problem along
// n = -d / r with left state i.  The limited middle state
//   u* = (z_l u_l + z_r u_r + beta^2 (p_l - p_r)) / (z_l + z_r),
//   p* = (p_l + p_r)/2 + beta/2 (z_r (u* - u_r) + z_l (u_l - u*)),
// z = rho c, beta = min(eta max((u_l - u_r) / cbar, 0), 1); the wave
// speeds u_l - c_l, u_r + c_r, or min/max estimates where those cross; at
// the fixed interface the upwind state when the fan is one-sided, else the
// star state on the side of u*'s sign,
//   rho*_K = rho_K (S_K - u_K) / (S_K - u*),
//   E*_K = ((S_K - u_K) E_K - p_K u_K + p* u*) / (S_K - u*),
// velocity u* n plus the mean tangential velocity.  With w = V_j (1-q/2)^3,
// G = (B_i + B_j) d and the row factor -cF:
//   drho/dt = -cF sum_j w rho_I (v_I . G),
//   dm/dt   = -cF sum_j w [rho_I v_I (v_I . G) + p_I G],
//   dE/dt   = -cF sum_j w (E_I + p_I) (v_I . G).
// A padding entry (the particle itself) has w = 0 and finite terms.
template <bool WRAP>
__device__ __forceinline__ void accumulate_pair_hllc(const EulerArgs& ea, const OwnState<2>& o, const NbrRec<2>& nb,
                                                     Kahan& sr, Kahan* sm, Kahan& se) {
    const float4 gj = nb.g0;  // (x, y, V, B00)
    const float Bs[3] = {o.B[0] + gj.w, o.B[1] + nb.g1.x, o.B[2] + nb.g1.y};
    const float4 pj = nb.pr;  // (rho, v_x, v_y, p)
    float d[2];
    d[0] = o.x[0] - gj.x;
    d[1] = o.x[1] - gj.y;
    if (WRAP) {
        d[0] = wrap(d[0], ea.L[0], ea.invL[0]);
        d[1] = wrap(d[1], ea.L[1], ea.invL[1]);
    }
    const float r2 = fmaf(d[0], d[0], d[1] * d[1]);
    const bool live = r2 > 0.f;
    const float rinv = live ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float tq = fmaf(ea.nhh, r2 * rinv, 1.f);  // 1 - q/2
    const float Vj = live ? gj.z : 0.f;
    const float w = (Vj * tq) * (tq * tq);
    const float G0 = fmaf(Bs[0], d[0], Bs[1] * d[1]);
    const float G1 = fmaf(Bs[1], d[0], Bs[2] * d[1]);
    const float n0 = -d[0] * rinv, n1 = -d[1] * rinv;
    const float ul = fmaf(o.v[0], n0, o.v[1] * n1);
    const float ur = fmaf(pj.y, n0, pj.z * n1);
    const float rhor = pj.x, pr = pj.w;
    const float cr = __builtin_amdgcn_sqrtf(ea.gamma * pr * fast_rcp(rhor));
    const float zr = rhor * cr;
    const float Er = fmaf(pr, ea.ig1, 0.5f * rhor * fmaf(pj.y, pj.y, pj.z * pj.z));
    float Sl = ul - o.c, Sr = ur + cr;
    const bool cross = Sl > Sr;
    Sl = cross ? fminf(ul - o.c, ur - cr) : Sl;
    Sr = cross ? fmaxf(ul + o.c, ur + cr) : Sr;
    const float izs = fast_rcp(o.z + zr);
    const float beta = __builtin_amdgcn_fmed3f(2.f * ea.eta_h * (ul - ur) * fast_rcp(o.c + cr), 0.f, 1.f);
    const float us = (fmaf(o.z, ul, zr * ur) + (beta * beta) * (o.p - pr)) * izs;
    const float ps = 0.5f * ((o.p + pr) + beta * fmaf(zr, us - ur, o.z * (ul - us)));
    // star state on the side of u*
    const bool left = us >= 0.f;
    const float rhoK = left ? o.rho : rhor, uK = left ? ul : ur, SK = left ? Sl : Sr;
    const float EK = left ? o.Et : Er, pK = left ? o.p : pr;
    const float den = fast_rcp(SK - us);
    float rhoI = rhoK * (SK - uK) * den;
    float EI = fmaf(SK - uK, EK, fmaf(ps, us, -pK * uK)) * den;
    float pI = ps;
    const float um = 0.5f * (ul + ur);
    float vI0 = fmaf(us - um, n0, 0.5f * (o.v[0] + pj.y));
    float vI1 = fmaf(us - um, n1, 0.5f * (o.v[1] + pj.z));
    // one-sided fans: the upwind state
    const bool upl = Sl >= 0.f, upr = !upl && Sr <= 0.f;
    rhoI = upl ? o.rho : (upr ? rhor : rhoI);
    pI = upl ? o.p : (upr ? pr : pI);
    EI = upl ? o.Et : (upr ? Er : EI);
    vI0 = upl ? o.v[0] : (upr ? pj.y : vI0);
    vI1 = upl ? o.v[1] : (upr ? pj.z : vI1);
    const float vG = fmaf(vI0, G0, vI1 * G1);
    const float rvG = rhoI * vG;
    accum(sr, w, rvG);
    accum(sm[0], w, fmaf(rvG, vI0, pI * G0));
    accum(sm[1], w, fmaf(rvG, vI1, pI * G1));
    accum(se, w, (EI + pI) * vG);
}

// Compressible primitive record (rho, v_x, v_y, p) of U = (rho, m_x, m_y, E).
__device__ __forceinline__ float4 primitive_hllc(const float4& u, float gm1) {
    const float inv = fast_rcp(u.x);
    const float vx = u.y * inv, vy = u.z * inv;
    return make_float4(u.x, vx, vy, gm1 * (u.w - 0.5f * fmaf(u.y, vx, u.z * vy)));
}

__global__ void k_pack_hllc(int32_t n, float gm1, const float4* __restrict__ sorted, const float* __restrict__ rho,
                            const float* __restrict__ mom, const float* __restrict__ E, float4* __restrict__ U,
                            float4* __restrict__ P) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = __float_as_int(sorted[s].w);
    const float4 u = make_float4(rho[i], mom[i], mom[(int64_t)n + i], E[i]);
    U[s] = u;
    P[s] = primitive_hllc(u, gm1);
}

__global__ void k_unpack_hllc(int32_t n, const float4* __restrict__ sorted, const float4* __restrict__ U,
                              float* __restrict__ rho, float* __restrict__ mom, float* __restrict__ E) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = __float_as_int(sorted[s].w);
    const float4 u = U[s];
    rho[i] = u.x;
    mom[i] = u.y;
    mom[(int64_t)n + i] = u.z;
    E[i] = u.w;
}

// Solver of the stage kernel: the weakly compressible rows with the
// linearised solver (EOS p = c^2 (rho - rho0)) or the compressible rows with
// the limited HLLC solver (ideal gas, 2-D).
enum Solver { SOL_LINEARISED = 0, SOL_HLLC = 1 };

template <int DIM, int SOL, bool WRAP>
__device__ __forceinline__ void pair_terms(const EulerArgs& ea, const OwnState<DIM>& o, const NbrRec<DIM>& nb,
                                           Kahan& sr, Kahan* sm, Kahan& se) {
    if constexpr (SOL == SOL_HLLC) accumulate_pair_hllc<WRAP>(ea, o, nb, sr, sm, se);
    else accumulate_pair<DIM, WRAP>(ea, o, nb, sr, sm);
}

enum RowMode { ROWS_CSR = 0, ROWS_ELL = 1, ROWS_ELL_BATCH = 2 };

// Batch mode: the column indices of a lane's E entries of row i.
template <int L, int E>
__device__ __forceinline__ void load_batch_cols(int32_t n, const int32_t* __restrict__ col, int32_t ell_S,
                                                int32_t i, int sub, int32_t* jb) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int32_t kk = sub + q * L;
        jb[q] = kk < ell_S ? ld32(col, (uint32_t)kk * (uint32_t)n + (uint32_t)i) : i;
    }
}

// One particle's row for lane `sub` of its group (batch mode: the lane's
// column indices in jb).  Every gather of the row is issued before the own
// record is waited on.
template <int DIM, int SOL, int STAGE, int L, int MODE, int E>
__device__ __forceinline__ void euler_row(int32_t n, const EulerArgs& ea, const int64_t* __restrict__ row_ptr,
                                          const int32_t* __restrict__ col, int32_t ell_S,
                                          const float4* __restrict__ geo0, const float4* __restrict__ geo1,
                                          const float2* __restrict__ geo2, const float4* U,
                                          const float4* __restrict__ P, const float4* U0, float4* Uout,
                                          float4* Pout, const float4* __restrict__ sorted,
                                          float* __restrict__ drho_dt, float* __restrict__ dmom_dt,
                                          float* __restrict__ dE_dt, int32_t i, int sub, const int32_t* jb) {
    NbrRec<DIM> self;
    gather_nbr<DIM>(i, geo0, geo1, geo2, P, self);
    // batch mode: every record of the lane's entries in flight at once
    NbrRec<DIM> nb[MODE == ROWS_ELL_BATCH && E > 0 ? E : 1];
    if (MODE == ROWS_ELL_BATCH) {
#pragma unroll
        for (int q = 0; q < E; ++q) gather_nbr<DIM>(jb[q], geo0, geo1, geo2, P, nb[q]);
    }
    // the stage update's inputs, loaded now so that their latency overlaps the row
    float4 ui = make_float4(0.f, 0.f, 0.f, 0.f), u0 = ui;
    if (STAGE != 0 && sub == 0) {
        ui = U[i];
        if (STAGE == 2) u0 = U0[i];
    }

    OwnState<DIM> o;
    const float4 gi = self.g0;
    o.x[0] = gi.x; o.x[1] = gi.y; o.x[2] = gi.z;
    if (DIM == 2) {
        o.B[0] = gi.w; o.B[1] = self.g1.x; o.B[2] = self.g1.y;
    } else {
        o.B[0] = self.g1.x; o.B[1] = self.g1.y; o.B[2] = self.g1.z; o.B[3] = self.g1.w;
        o.B[4] = self.g2.x; o.B[5] = self.g2.y;
    }
    const float4 pi4 = self.pr;
    // periodic wrap only in waves with a particle near a periodic face
    bool near = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (ea.invL[a] != 0.f) {
            const float off = o.x[a] - ea.lo[a];
            near = near || off < ea.margin || ea.L[a] - off < ea.margin;
        }
    }
    const bool wrap_wave = __any(near);
    if constexpr (SOL == SOL_HLLC) {
        o.v[0] = pi4.y; o.v[1] = pi4.z; o.v[2] = 0.f;
        o.rho = pi4.x;
        o.p = pi4.w;
        o.c = __builtin_amdgcn_sqrtf(ea.gamma * o.p * fast_rcp(o.rho));
        o.z = o.rho * o.c;
        o.Et = fmaf(o.p, ea.ig1, 0.5f * o.rho * fmaf(o.v[0], o.v[0], o.v[1] * o.v[1]));
    } else {
        o.v[0] = pi4.y; o.v[1] = pi4.z; o.v[2] = pi4.w;
        o.p2 = fmaf(ea.c2x2, pi4.x, ea.c2x2poff);
        o.crho = ea.c * ((ea.rho_ref + pi4.x) + ea.rho_ref);
    }

    Kahan sr, sm[DIM], se;
    sr.init();
    se.init();
#pragma unroll
    for (int a = 0; a < DIM; ++a) sm[a].init();

    if (MODE == ROWS_ELL_BATCH) {
        if (wrap_wave) {
#pragma unroll
            for (int q = 0; q < E; ++q) pair_terms<DIM, SOL, true>(ea, o, nb[q], sr, sm, se);
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) pair_terms<DIM, SOL, false>(ea, o, nb[q], sr, sm, se);
        }
    } else {
        int64_t k, e, stride;
        if (MODE == ROWS_ELL) {
            k = (int64_t)sub * n + i;
            stride = n;
            e = (int64_t)ell_S * n;
        } else {
            k = row_ptr[i] + sub;
            stride = 1;
            e = row_ptr[i + 1];
        }
        NbrRec<DIM> cur, nxt;
        {
            const int32_t j0 = k < e ? col[k] : i;
            gather_nbr<DIM>(j0, geo0, geo1, geo2, P, cur);
        }
        int32_t jn1 = k + L * stride < e ? col[k + L * stride] : i;
        while (k < e) {
            gather_nbr<DIM>(jn1, geo0, geo1, geo2, P, nxt);
            jn1 = k + 2 * L * stride < e ? col[k + 2 * L * stride] : i;
            k += L * stride;
            if (wrap_wave) pair_terms<DIM, SOL, true>(ea, o, cur, sr, sm, se);
            else pair_terms<DIM, SOL, false>(ea, o, cur, sr, sm, se);
            cur = nxt;
        }
    }
    // R = (rho or drho, m, E or m_z) rates
    float R[4];
    if constexpr (SOL == SOL_HLLC) {
        R[0] = ea.fh * group_sum<L>(sr);
        R[1] = ea.fh * group_sum<L>(sm[0]);
        R[2] = ea.fh * group_sum<L>(sm[1]);
        R[3] = ea.fh * group_sum<L>(se);
    } else {
        R[0] = ea.fr * group_sum<L>(sr);
#pragma unroll
        for (int a = 0; a < DIM; ++a) R[1 + a] = ea.fm * group_sum<L>(sm[a]);
        if (DIM == 2) R[3] = 0.f;
    }
    constexpr bool R4 = DIM == 3 || SOL == SOL_HLLC;  // the fourth record component evolves
    if (sub != 0) return;
    if (STAGE == 0) {
        const int32_t ic = __float_as_int(sorted[i].w);
        drho_dt[ic] = R[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) dmom_dt[(int64_t)a * n + ic] = R[1 + a];
        if (SOL == SOL_HLLC) dE_dt[ic] = R[3];
        return;
    }
    float4 un;
    if (STAGE == 1) {
        un = make_float4(ui.x + ea.dt * R[0], ui.y + ea.dt * R[1], ui.z + ea.dt * R[2],
                         R4 ? ui.w + ea.dt * R[3] : 0.f);
    } else {
        un = make_float4(0.5f * (u0.x + (ui.x + ea.dt * R[0])), 0.5f * (u0.y + (ui.y + ea.dt * R[1])),
                         0.5f * (u0.z + (ui.z + ea.dt * R[2])),
                         R4 ? 0.5f * (u0.w + (ui.w + ea.dt * R[3])) : 0.f);
    }
    Uout[i] = un;
    if constexpr (SOL == SOL_HLLC) Pout[i] = primitive_hllc(un, ea.gm1);
    else Pout[i] = primitive<DIM>(un, ea.rho_ref);
}

// One lane group of L lanes per particle.  STAGE 0: write rates; 1: Uout =
// U + dt R(U); 2: Uout = (U0 + U + dt R(U)) / 2; stages 1 and 2 also write
// Pout, the primitive record of Uout.  Uout / Pout may alias U0 / the own
// records of the stage input: each particle's records are read and written
// only by its own lane group, and neighbours are gathered from P, which a
// stage never writes in place.  Lane `sub` of the group takes the row
// entries sub, sub + L, ...; the lanes' partial sums are combined by
// group_sum and lane 0 of the group writes the result.
//   ROWS_CSR / ROWS_ELL: a software pipeline over the row: the records of
//     the next entry are gathered and the column index after it loaded
//     before the current pair is evaluated.
//   ROWS_ELL_BATCH: the lane's E entries are loaded at once (all column
//     indices, then all records) and then evaluated (short rows, where a
//     pipeline would be too shallow to cover the memory latency).
// Entries past the end of a row use the particle itself (zero weight).
// Blocks run in XCD-contiguous order; whole groups leave together.
template <int DIM, int SOL, int STAGE, int L, int MODE, int E>
__global__ void __launch_bounds__(BLK) k_euler(int32_t n, EulerArgs ea, const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, int32_t ell_S,
                                               const float4* __restrict__ geo0,
                                               const float4* __restrict__ geo1, const float2* __restrict__ geo2,
                                               const float4* U, const float4* __restrict__ P, const float4* U0,
                                               float4* Uout, float4* Pout, const float4* __restrict__ sorted,
                                               float* __restrict__ drho_dt, float* __restrict__ dmom_dt,
                                               float* __restrict__ dE_dt) {
    const int32_t blk = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int sub = (int)(threadIdx.x % L);
    const int32_t i = blk * (BLK / L) + (int32_t)(threadIdx.x / L);
    if (i >= n) return;
    int32_t jb[E > 0 ? E : 1];
    if (MODE == ROWS_ELL_BATCH) load_batch_cols<L, E>(n, col, ell_S, i, sub, jb);
    euler_row<DIM, SOL, STAGE, L, MODE, E>(n, ea, row_ptr, col, ell_S, geo0, geo1, geo2, U, P, U0, Uout,
                                               Pout, sorted, drho_dt, dmom_dt, dE_dt, i, sub, jb);
}

// ------------------------------------------------------------------ 3-D stage on packed records
// In 3-D the per-particle stage gathers each neighbour from one 64-byte
// record (one cache-line half) in cell-sorted order:
//   q0 = (x, y, z, V), q1 = (B00, B01, B02, B11), q2 = (B12, B22, 0, 0),
//   q3 = (2 p, v_x, v_y, v_z),  2 p = 2 c^2 (drho + rho_ref - rho0),
// so that a pair needs no per-partner arithmetic for the pressure (and
// reads 56 bytes of the record).  Two record sets carry the stage input and output; geometry
// is written into both when the state is packed, and a stage writes only
// the q3 quad of its output (with the conserved record U).

// q3 of a conserved record u = (drho, m): (2 p, v) with 2 p = 2 c^2 (drho +
// rho_ref - rho0) and v = m / (rho_ref + drho).
__device__ __forceinline__ float4 state_quad3(const EulerArgs& ea, const float4& u) {
    const float inv = fast_rcp(ea.rho_ref + u.x);
    return make_float4(fmaf(ea.c2x2, u.x, ea.c2x2poff), u.y * inv, u.z * inv, u.w * inv);
}

// Records of the stage input from the caller's state (gathered at the caller
// index of each sorted slot) and the cached geometry: conserved U, and the
// full records in both record sets.
__global__ void k_pack3(int32_t n, EulerArgs ea, const float4* __restrict__ sorted, const float* __restrict__ drho,
                        const float* __restrict__ mom, const float4* __restrict__ geo0,
                        const float4* __restrict__ geo1, const float2* __restrict__ geo2, float4* __restrict__ U,
                        float4* __restrict__ Ra, float4* __restrict__ Rb) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t i = __float_as_int(sorted[s].w);
    const float4 u = make_float4(drho[i], mom[i], mom[(int64_t)n + i], mom[2 * (int64_t)n + i]);
    U[s] = u;
    const float4 g0 = geo0[s], g1 = geo1[s];
    const float2 g2 = geo2[s];
    const float4 q2 = make_float4(g2.x, g2.y, 0.f, 0.f);
    const float4 q3 = state_quad3(ea, u);
    const int64_t b = 4 * (int64_t)s;
    Ra[b] = g0; Ra[b + 1] = g1; Ra[b + 2] = q2; Ra[b + 3] = q3;
    Rb[b] = g0; Rb[b + 1] = g1; Rb[b + 2] = q2; Rb[b + 3] = q3;
}

struct Rec3 {
    float4 q0, q1, q2, q3;
};

__device__ __forceinline__ void gather3(const float4* __restrict__ R, int32_t j, Rec3& r) {
    const uint32_t b = (uint32_t)j << 2;
    r.q0 = ld32(R, b);
    r.q1 = ld32(R, b + 1u);
    r.q2 = ld32(R, b + 2u);
    r.q3 = ld32(R, b + 3u);
}

// j, made to depend on the pair sum just updated (an empty asm statement
// emits no instruction): the next record's loads then stay after the pair
// that frees its registers instead of being hoisted above it (which would
// need a register set per record in flight).
__device__ __forceinline__ int32_t after(int32_t j, const Kahan& k) {
    asm volatile("" : "+v"(j) : "v"(k.s), "v"(k.c));
    return j;
}

// v, required in registers at this point (an empty asm statement that reads
// it: the loads that produce it are complete here).
__device__ __forceinline__ void held(const float4& v) {
    asm volatile("" : : "v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

struct Own3 {
    float x[3], B[6], v[3];
    float p2;     // 2 p_i
    float crho;   // c rho_i + c rho0 (so that c (rho_i + rho_j) = crho + 2 p_j / (2 c))
    float ktrB;   // k tr B_i, k = -4 mu / d
};

// One pair (i, j) of Eq. (19) in 3-D with the corrected gradient (Eq. 28)
// and the limited linearised Riemann solution (Eqs. 26-27): the terms of
// accumulate_pair, with 2 p_j read from the partner's record, tr B_j summed
// from its B entries and c (rho_i + rho_j) = (c rho_i + c rho0) + 2 p_j /
// (2 c).  The row's
// pairs come two at a time: the first of two opens the compensated
// additions (OPEN), the second closes them.
template <bool WRAP, bool OPEN>
__device__ __forceinline__ void pair3(const EulerArgs& ea, const Own3& o, const Rec3& nb, Kahan& sr, Kahan* sm) {
    float d[3], dv[3];
    d[0] = o.x[0] - nb.q0.x;
    d[1] = o.x[1] - nb.q0.y;
    d[2] = o.x[2] - nb.q0.z;
    if (WRAP) {
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] = wrap(d[a], ea.L[a], ea.invL[a]);
    }
    dv[0] = o.v[0] - nb.q3.y;
    dv[1] = o.v[1] - nb.q3.z;
    dv[2] = o.v[2] - nb.q3.w;
    const float r2 = fmaf(d[0], d[0], fmaf(d[1], d[1], d[2] * d[2]));
    const float dvd = fmaf(dv[0], d[0], fmaf(dv[1], d[1], dv[2] * d[2]));
    const bool live = r2 > 0.f;
    const float rinv = live ? __builtin_amdgcn_rsqf(r2) : 0.f;
    const float tq = fmaf(ea.nhh, r2 * rinv, 1.f);  // 1 - q/2
    const float Vj = live ? nb.q0.w : 0.f;
    const float w = (Vj * tq) * (tq * tq);
    const float B0 = o.B[0] + nb.q1.x, B1 = o.B[1] + nb.q1.y, B2 = o.B[2] + nb.q1.z;
    const float B3 = o.B[3] + nb.q1.w, B4 = o.B[4] + nb.q2.x, B5 = o.B[5] + nb.q2.y;
    const float G0 = fmaf(B0, d[0], fmaf(B1, d[1], B2 * d[2]));
    const float G1 = fmaf(B1, d[0], fmaf(B3, d[1], B4 * d[2]));
    const float G2 = fmaf(B2, d[0], fmaf(B4, d[1], B5 * d[2]));
    const float a = dvd * rinv;
    const float beta = __builtin_amdgcn_fmed3f(ea.nec * a, 0.f, 1.f);
    const float pj2 = nb.q3.x;
    const float crho = fmaf(pj2, ea.inv2c, o.crho);
    const float du2 = ((beta * beta) * (o.p2 - pj2)) * fast_rcp(crho);
    const float p4 = fmaf(-(beta * crho), a, o.p2 + pj2);
    const float rhostar = fmaf(p4, ea.qc2inv, ea.rho0);
    const float dn = du2 * rinv;
    const float vs0 = fmaf(-dn, d[0], o.v[0] + nb.q3.y);
    const float vs1 = fmaf(-dn, d[1], o.v[1] + nb.q3.z);
    const float vs2 = fmaf(-dn, d[2], o.v[2] + nb.q3.w);
    const float vg2 = fmaf(vs0, G0, fmaf(vs1, G1, vs2 * G2));
    const float rh = rhostar * vg2;
    const float kv = fmaf(ea.kmu, (nb.q1.x + nb.q1.w) + nb.q2.y, o.ktrB);
    const float xm0 = fmaf(rh, vs0, fmaf(p4, G0, kv * dv[0]));
    const float xm1 = fmaf(rh, vs1, fmaf(p4, G1, kv * dv[1]));
    const float xm2 = fmaf(rh, vs2, fmaf(p4, G2, kv * dv[2]));
    if (OPEN) {
        sr.open(w, rh);
        sm[0].open(w, xm0);
        sm[1].open(w, xm1);
        sm[2].open(w, xm2);
    } else {
        sr.close(w, rh);
        sm[0].close(w, xm0);
        sm[1].close(w, xm1);
        sm[2].close(w, xm2);
    }
}

// The lane's entries t = 0 .. m-1 of row i (entry t at e0 + t es), taken in
// chunks of M pairs over a wave-uniform count mu >= m (entries past the
// lane's end stand for the particle itself: a zero-weight pair, so every
// lane runs the same straight-line code).  A chunk's column indices are
// loaded first (no gather then waits behind an index load issued after
// it), then its records are gathered two ahead of the pair being evaluated,
// into two register sets refilled in turn (no register copies); scheduling
// barriers keep each gather where it is issued.  M is even: the pairs enter
// the compensated sums two at a time.
template <bool WRAP, int M>
__device__ __forceinline__ void row3(const EulerArgs& ea, const Own3& o, const float4* __restrict__ R,
                                     const int32_t* __restrict__ col, int32_t i, uint32_t e0, uint32_t es, int32_t m,
                                     int32_t mu, Kahan& sr, Kahan* sm) {
    for (int32_t base = 0; base < mu; base += M) {
        int32_t jb[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const int32_t t = base + q < m ? base + q : m - 1;
            const int32_t v = ld32(col, m > 0 ? e0 + (uint32_t)t * es : 0u);  // always an entry of the array
            jb[q] = base + q < m ? v : i;
        }
        Rec3 A, B;
        gather3(R, jb[0], A);
        gather3(R, jb[1], B);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < M; q += 2) {
            pair3<WRAP, true>(ea, o, A, sr, sm);
            if (q + 2 < M) gather3(R, after(jb[q + 2], sr), A);
            __builtin_amdgcn_sched_barrier(0);
            pair3<WRAP, false>(ea, o, B, sr, sm);
            if (q + 3 < M) gather3(R, after(jb[q + 3], sr), B);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// One lane group of L lanes per particle (sorted slot i).  STAGE 0 writes
// the rates at the caller index; 1: Uout = U + dt R(U); 2: Uout = (U0 + U +
// dt R(U)) / 2, and both write q3 of Rout for Uout.  Rout may be the
// record set of U0: each particle's records are read and written only by
// its own group, and neighbours are gathered from R, which a stage never
// writes.  ELL rows: entry k of slot i at col[k n + i] (k < S); CSR rows:
// rp.  Lane sub takes entries sub, sub + L, ...
template <int STAGE, int L, bool ELL, int M>
__global__ void __launch_bounds__(BLK) k_euler3(int32_t n, EulerArgs ea, const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col, int32_t S,
                                                const float4* __restrict__ R, float4* Rout, const float4* U,
                                                const float4* U0, float4* Uout, const float4* __restrict__ sorted,
                                                float* __restrict__ drho_dt, float* __restrict__ dmom_dt) {
    const int32_t blk = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int sub = (int)(threadIdx.x % L);
    const int32_t ig = blk * (BLK / L) + (int32_t)(threadIdx.x / L);
    // every lane of the wave stays to the end (the wave-wide maximum below
    // reads all of them); groups past the last particle take its row and
    // write nothing
    const bool valid = ig < n;
    const int32_t i = valid ? ig : n - 1;
    uint32_t e0, es;
    int32_t m, mu;
    if (ELL) {
        e0 = (uint32_t)sub * (uint32_t)n + (uint32_t)i;
        es = (uint32_t)L * (uint32_t)n;
        m = (S - sub + L - 1) / L;
        mu = (S + L - 1) / L;
    } else {
        const int64_t b = rp[i], e = rp[i + 1];
        e0 = (uint32_t)b + (uint32_t)sub;
        es = (uint32_t)L;
        m = (int32_t)((e - b - sub + L - 1) / L);
        m = m > 0 ? m : 0;
        mu = m;
#pragma unroll
        for (int k = 1; k < 64; k <<= 1) mu = max(mu, __shfl_xor(mu, k, 64));  // the wave's longest share
    }
    Rec3 self;
    gather3(R, i, self);
    float4 ui = make_float4(0.f, 0.f, 0.f, 0.f), u0 = ui;
    if (STAGE != 0 && sub == 0) {
        ui = U[i];
        if (STAGE == 2) u0 = U0[i];
    }
    Own3 o;
    o.x[0] = self.q0.x; o.x[1] = self.q0.y; o.x[2] = self.q0.z;
    o.B[0] = self.q1.x; o.B[1] = self.q1.y; o.B[2] = self.q1.z; o.B[3] = self.q1.w;
    o.B[4] = self.q2.x; o.B[5] = self.q2.y;
    o.ktrB = ea.kmu * ((self.q1.x + self.q1.w) + self.q2.y);
    o.p2 = self.q3.x;
    o.v[0] = self.q3.y; o.v[1] = self.q3.z; o.v[2] = self.q3.w;
    o.crho = fmaf(o.p2, ea.inv2c, ea.crho0x2);
    // periodic wrap only in waves with a particle near a periodic face
    bool near = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (ea.invL[a] != 0.f) {
            const float off = o.x[a] - ea.lo[a];
            near = near || off < ea.margin || ea.L[a] - off < ea.margin;
        }
    }
    Kahan sr, sm[3];
    sr.init();
#pragma unroll
    for (int a = 0; a < 3; ++a) sm[a].init();
    if (__any(near)) row3<true, M>(ea, o, R, col, i, e0, es, m, mu, sr, sm);
    else row3<false, M>(ea, o, R, col, i, e0, es, m, mu, sr, sm);
    float Rt[4];
    Rt[0] = ea.fr * group_sum<L>(sr);
#pragma unroll
    for (int a = 0; a < 3; ++a) Rt[1 + a] = ea.fm * group_sum<L>(sm[a]);
    if (sub != 0 || !valid) return;
    if (STAGE == 0) {
        const int32_t ic = __float_as_int(sorted[i].w);
        drho_dt[ic] = Rt[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) dmom_dt[(int64_t)a * n + ic] = Rt[1 + a];
        return;
    }
    float4 un;
    if (STAGE == 1) {
        un = make_float4(ui.x + ea.dt * Rt[0], ui.y + ea.dt * Rt[1], ui.z + ea.dt * Rt[2], ui.w + ea.dt * Rt[3]);
    } else {
        un = make_float4(0.5f * (u0.x + (ui.x + ea.dt * Rt[0])), 0.5f * (u0.y + (ui.y + ea.dt * Rt[1])),
                         0.5f * (u0.z + (ui.z + ea.dt * Rt[2])), 0.5f * (u0.w + (ui.w + ea.dt * Rt[3])));
    }
    Uout[i] = un;
    Rout[4 * (int64_t)i + 3] = state_quad3(ea, un);
}

// ------------------------------------------------------------------ record windows
// The 3-D stage over neighbour windows (built by sph_windows_prepare): a
// workgroup copies the records of its block's window into LDS once and its
// pairs then read them there instead of gathering each neighbour through
// the vector cache.

// Record k of the window from the LDS planes (plane q holds quad q of every
// record: a 16-byte read per quad, consecutive records in consecutive bank
// groups).
template <int HC>
__device__ __forceinline__ void wread(const float4* W, uint32_t k, Rec3& r) {
    r.q0 = W[k];
    r.q1 = W[HC + k];
    r.q2 = W[2 * HC + k];
    r.q3 = W[3 * HC + k];
}

// The same from the byte offset 16 k of the record in its plane.
template <int HC>
__device__ __forceinline__ void wread_b(const float4* W, uint32_t b, Rec3& r) {
    const char* w = reinterpret_cast<const char*>(W) + b;
    r.q0 = *reinterpret_cast<const float4*>(w);
    r.q1 = *reinterpret_cast<const float4*>(w + 16 * HC);
    r.q2 = *reinterpret_cast<const float4*>(w + 32 * HC);
    r.q3 = *reinterpret_cast<const float4*>(w + 48 * HC);
}

// row3 over the window: the lane's entries are the byte offsets (16 times
// the window position) of its neighbours' records, the records come from
// LDS (the pair order, and so every sum, is that of row3).  The lane's
// entries of chunk c sit together (M 16-bit values from word at0 + c cs),
// and the rows are padded to a whole number of chunks per lane.
template <bool WRAP, int M, int HC>
__device__ __forceinline__ void row3w(const EulerArgs& ea, const Own3& o, const float4* W,
                                      const uint16_t* __restrict__ colw, uint32_t at0, uint32_t cs, int32_t nchunk,
                                      Kahan& sr, Kahan* sm) {
    for (int32_t c = 0; c < nchunk; ++c) {
        uint32_t w[M / 2];
        load_chunk<M>(colw, at0 + (uint32_t)c * cs, w);
        Rec3 A, B;
        wread_b<HC>(W, w[0] & 0xffffu, A);
        wread_b<HC>(W, w[0] >> 16, B);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < M; q += 2) {
            pair3<WRAP, true>(ea, o, A, sr, sm);
            if (q + 2 < M) wread_b<HC>(W, (uint32_t)after((int32_t)(w[q / 2 + 1] & 0xffffu), sr), A);
            __builtin_amdgcn_sched_barrier(0);
            pair3<WRAP, false>(ea, o, B, sr, sm);
            if (q + 3 < M) wread_b<HC>(W, (uint32_t)after((int32_t)(w[q / 2 + 1] >> 16), sr), B);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// TwoSum merge of a compensated partial (hi, lo) with another (ohi, olo);
// the error term of TwoSum is exact, so the result does not depend on which
// operand is first.
__device__ __forceinline__ void merge_pair(float& hi, float& lo, float ohi, float olo) {
    const float s = hi + ohi;
    const float bp = s - hi;
    const float e = (hi - (s - bp)) + (ohi - bp);
    lo = (lo + olo) + e;
    hi = s;
}

// The four compensated sums k[0..3] of the four lanes of a group, reduced
// and distributed: the lane with sub = b0 + 2 b1 returns the total of sum
// 2 b0 + b1.  The lanes merge the same pairs as group_sum<4> (first lanes x
// and x ^ 1, then x and x ^ 2), each lane carrying half the sums at the
// first level and one at the second, so every total has the bits of
// group_sum<4>'s.
__device__ __forceinline__ float group_sum4_spread(const Kahan* k, int sub) {
    const bool b0 = (sub & 1) != 0, b1 = (sub & 2) != 0;
    float kh0 = b0 ? k[2].s : k[0].s, kl0 = b0 ? -k[2].c : -k[0].c;
    float kh1 = b0 ? k[3].s : k[1].s, kl1 = b0 ? -k[3].c : -k[1].c;
    const float sh0 = b0 ? k[0].s : k[2].s, sl0 = b0 ? -k[0].c : -k[2].c;
    const float sh1 = b0 ? k[1].s : k[3].s, sl1 = b0 ? -k[1].c : -k[3].c;
    merge_pair(kh0, kl0, lane_xor(sh0, 1), lane_xor(sl0, 1));
    merge_pair(kh1, kl1, lane_xor(sh1, 1), lane_xor(sl1, 1));
    float kh = b1 ? kh1 : kh0, kl = b1 ? kl1 : kl0;
    const float sh = b1 ? kh0 : kh1, sl = b1 ? kl0 : kl1;
    merge_pair(kh, kl, lane_xor(sh, 2), lane_xor(sl, 2));
    return kh + kl;
}

// k_euler3 with the neighbour records read from the workgroup's window in
// LDS (fixed-stride rows only, four lanes per particle).  Workgroup blk of NT
// threads takes block blk of P = NT / 4 slots; its window (at most HC
// records) is copied from R first.  Rows of Sp entries (Sp / 4 a multiple of
// M).  The group's four sums end on its four lanes (group_sum4_spread) and
// each lane finishes one component: lane sub takes component
// 2 (sub & 1) + (sub >> 1) of (drho, m).  Results are bit-identical to
// k_euler3's.
// Waves per SIMD when as many window workgroups are resident as a CU's
// 160 KB of LDS holds; the register budget is capped to match (with 512
// threads and 768-record windows: three workgroups, six waves per SIMD, at
// most 80 VGPRs).
template <int HC, int NT>
constexpr int window_waves_per_simd() { return 163840 / (64 * HC) * (NT / 64) / 4; }

template <int STAGE, int M, int HC, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(window_waves_per_simd<HC, NT>())))
k_euler3w(int32_t n, EulerArgs ea, const uint16_t* __restrict__ colw,
                                                int32_t Sp, const int32_t* __restrict__ woff,
                                                const int32_t* __restrict__ wlist, const float4* __restrict__ R,
                                                float4* Rout, const float4* U, const float4* U0, float4* Uout,
                                                const float4* __restrict__ sorted, float* __restrict__ drho_dt,
                                                float* __restrict__ dmom_dt) {
    constexpr int L = 4;
    __shared__ float4 W[4 * HC];
    const int32_t blk = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x);
    const int32_t w0 = woff[blk], wn = woff[blk + 1] - w0;
    {
        // a thread per record, at most KC records each: the slot indices
        // are loaded first, then the records, then written to LDS, so the
        // copy waits on two memory latencies, not 2 KC.  Threads past the
        // window's end load its last record again (every window holds the
        // block's own slots, so it is never empty) and write nothing.
        constexpr int KC = (HC + NT - 1) / NT;
        uint32_t b[KC];
#pragma unroll
        for (int r = 0; r < KC; ++r) b[r] = (uint32_t)min((int32_t)threadIdx.x + r * NT, wn - 1);
#pragma unroll
        for (int r = 0; r < KC; ++r) b[r] = (uint32_t)wlist[w0 + (int32_t)b[r]] << 2;
        float4 a[KC][4];
#pragma unroll
        for (int r = 0; r < KC; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[r][q] = ld32(R, b[r] + (uint32_t)q);
        }
        // (the records are taken here, so that no load is moved into the
        // guarded writes below, behind the first of them)
#pragma unroll
        for (int r = 0; r < KC; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) held(a[r][q]);
        }
#pragma unroll
        for (int r = 0; r < KC; ++r) {
            const int32_t k = (int32_t)threadIdx.x + r * NT;
            if (k < wn) {
#pragma unroll
                for (int q = 0; q < 4; ++q) W[q * HC + k] = a[r][q];
            }
        }
    }
    const int sub = (int)(threadIdx.x % L);
    const int comp = 2 * (sub & 1) + (sub >> 1);
    const int32_t lp = (int32_t)(threadIdx.x / L);
    const int32_t ig = blk * (NT / L) + lp;
    const bool valid = ig < n;
    const int32_t i = valid ? ig : n - 1;
    const uint32_t self = (uint32_t)(i - blk * (NT / L));
    // chunk c of the lane's entries: words ((c n + i) L + sub) M / 2 ..
    const uint32_t at0 = ((uint32_t)i * L + (uint32_t)sub) * (uint32_t)(M / 2);
    const uint32_t cs = (uint32_t)n * L * (uint32_t)(M / 2);
    const int32_t nchunk = Sp / (L * M);
    float uc = 0.f, u0c = 0.f;
    if (STAGE != 0) {
        uc = reinterpret_cast<const float*>(U)[4 * (int64_t)i + comp];
        if (STAGE == 2) u0c = reinterpret_cast<const float*>(U0)[4 * (int64_t)i + comp];
    }
    __syncthreads();
    Rec3 me;
    wread<HC>(W, self, me);
    Own3 o;
    o.x[0] = me.q0.x; o.x[1] = me.q0.y; o.x[2] = me.q0.z;
    o.B[0] = me.q1.x; o.B[1] = me.q1.y; o.B[2] = me.q1.z; o.B[3] = me.q1.w;
    o.B[4] = me.q2.x; o.B[5] = me.q2.y;
    o.ktrB = ea.kmu * ((me.q1.x + me.q1.w) + me.q2.y);
    o.p2 = me.q3.x;
    o.v[0] = me.q3.y; o.v[1] = me.q3.z; o.v[2] = me.q3.w;
    o.crho = fmaf(o.p2, ea.inv2c, ea.crho0x2);
    bool near = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (ea.invL[a] != 0.f) {
            const float off = o.x[a] - ea.lo[a];
            near = near || off < ea.margin || ea.L[a] - off < ea.margin;
        }
    }
    Kahan ks[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ks[a].init();
    if (__any(near)) row3w<true, M, HC>(ea, o, W, colw, at0, cs, nchunk, ks[0], ks + 1);
    else row3w<false, M, HC>(ea, o, W, colw, at0, cs, nchunk, ks[0], ks + 1);
    const float Rc = (comp == 0 ? ea.fr : ea.fm) * group_sum4_spread(ks, sub);
    if (STAGE == 0) {
        if (!valid) return;
        const int32_t ic = __float_as_int(sorted[i].w);
        if (comp == 0) drho_dt[ic] = Rc;
        else dmom_dt[(int64_t)(comp - 1) * n + ic] = Rc;
        return;
    }
    float unc;
    if (STAGE == 1) unc = uc + ea.dt * Rc;
    else unc = 0.5f * (u0c + (uc + ea.dt * Rc));
    // the density deviation sits on the group's first lane (component 0)
    const float dr = quad_first(unc);
    if (!valid) return;
    reinterpret_cast<float*>(Uout)[4 * (int64_t)i + comp] = unc;
    const float q3c = comp == 0 ? fmaf(ea.c2x2, unc, ea.c2x2poff) : unc * fast_rcp(ea.rho_ref + dr);
    reinterpret_cast<float*>(Rout)[16 * (int64_t)i + 12 + comp] = q3c;
}

EulerArgs make_args(const sph_ctx* c, const sph_euler_params* p) {
    EulerArgs a{};
    a.c = (float)p->c;
    a.hc = (float)(0.5 * p->c);
    a.c2 = (float)(p->c * p->c);
    a.c2inv = (float)(1.0 / (p->c * p->c));
    a.rho0 = (float)p->rho0;
    a.rho_ref = (float)p->rho_ref;
    a.poff = (float)(p->rho_ref - p->rho0);
    a.eta_c = (float)(p->eta / p->c);
    a.mu_tr = (float)(2.0 * p->mu / c->dim);
    a.dt = (float)p->dt;
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, c->dim, c->dom.h);
    a.hinv = kc.hinv;
    a.cFh = 0.5f * kc.cF;
    a.nhh = -0.5f * kc.hinv;
    a.c2x2 = (float)(2.0 * p->c * p->c);
    a.c2x2poff = (float)(2.0 * p->c * p->c * (p->rho_ref - p->rho0));
    a.nec = (float)(-p->eta / p->c);
    a.qc2inv = (float)(0.25 / (p->c * p->c));
    a.kmu = (float)(-4.0 * p->mu / c->dim);
    a.fr = (float)(-0.5 * (double)kc.cF);
    a.fm = (float)(-0.25 * (double)kc.cF);
    a.inv2c = (float)(0.5 / p->c);
    a.crho0x2 = (float)(2.0 * p->c * p->rho0);
    for (int ax = 0; ax < 3; ++ax) {
        a.L[ax] = c->box.L[ax];
        a.invL[ax] = c->box.periodic[ax] ? (float)(1.0 / c->box.Ld[ax]) : 0.f;
        a.lo[ax] = c->box.lo[ax];
    }
    a.margin = (float)(c->rc * 1.001);
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
    if (c->n >= (1 << 28))
        return sph_fail(c, SPH_ERR_ARG, "%s: %d particles exceed the 2^28 limit of the gathers", who, c->n);
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
    float* de;  // compressible rows: dE/dt (stage 0)
};

template <int DIM, int SOL, int STAGE, int L, int MODE, int E>
void launch_k(sph_ctx* c, const EulerArgs& ea, const StageIO& io) {
    const bool ell = MODE != ROWS_CSR;
    const dim3 grid(grid_for(c->n, BLK / L));
    const int64_t* rp = ell ? nullptr : c->rp_s.as<int64_t>();
    const int32_t* col = ell ? c->colE.as<int32_t>() : c->col_s.as<int32_t>();
    const int32_t S = ell ? c->ell_S : 0;
    hipLaunchKernelGGL((k_euler<DIM, SOL, STAGE, L, MODE, E>), grid, dim3(BLK), 0, c->stream, c->n, ea, rp, col, S,
                       c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), io.U, io.P, io.U0, io.Uout,
                       io.Pout, c->sorted.as<float4>(), io.dr, io.dm, io.de);
}

template <int DIM, int SOL, int STAGE, int L>
void launch_l(sph_ctx* c, const EulerArgs& ea, const StageIO& io) {
    if (c->ell_state == 1) launch_k<DIM, SOL, STAGE, L, ROWS_ELL, 0>(c, ea, io);
    else launch_k<DIM, SOL, STAGE, L, ROWS_CSR, 0>(c, ea, io);
}

// Batched short rows: L lanes per particle and E = ceil(S / L) entries per
// lane (at most 6, 5 or 4 for 2, 4 or 8 lanes).  Returns false when the rows
// are too long for a batch.
template <int DIM, int SOL, int STAGE>
bool launch_batch(sph_ctx* c, const EulerArgs& ea, const StageIO& io, int L) {
    const int E = (c->ell_S + L - 1) / L;
    if (L == 2) {
        if (E <= 4) launch_k<DIM, SOL, STAGE, 2, ROWS_ELL_BATCH, 4>(c, ea, io);
        else if (E == 5) launch_k<DIM, SOL, STAGE, 2, ROWS_ELL_BATCH, 5>(c, ea, io);
        else if (E == 6) launch_k<DIM, SOL, STAGE, 2, ROWS_ELL_BATCH, 6>(c, ea, io);
        else return false;
    } else if (L == 4) {
        if (E <= 2) launch_k<DIM, SOL, STAGE, 4, ROWS_ELL_BATCH, 2>(c, ea, io);
        else if (E == 3) launch_k<DIM, SOL, STAGE, 4, ROWS_ELL_BATCH, 3>(c, ea, io);
        else if (E == 4) launch_k<DIM, SOL, STAGE, 4, ROWS_ELL_BATCH, 4>(c, ea, io);
        else if (E == 5) launch_k<DIM, SOL, STAGE, 4, ROWS_ELL_BATCH, 5>(c, ea, io);
        else return false;
    } else if (L == 8) {
        if (E <= 2) launch_k<DIM, SOL, STAGE, 8, ROWS_ELL_BATCH, 2>(c, ea, io);
        else if (E == 3) launch_k<DIM, SOL, STAGE, 8, ROWS_ELL_BATCH, 3>(c, ea, io);
        else if (E == 4) launch_k<DIM, SOL, STAGE, 8, ROWS_ELL_BATCH, 4>(c, ea, io);
        else return false;
    } else {
        return false;
    }
    return true;
}

// Lanes per particle for the batched rows: 2 when six entries per lane
// cover the row, else 4 when five do (measured on the 2-D Taylor-Green rows:
// rows of 12 take 12.9 us per launch on 2 lanes, 13.7-14.3 on 4 -- the two
// lanes' records take 110 VGPRs, but the per-particle work and the lane
// combination are shared by half as many lanes; rows of 20 take 19.1 us on
// 4 batched lanes against 20.6 pipelined; with 8 lanes the pipelined loop is
// faster).  Below 2^15 particles two lanes give fewer than 1,024 waves and
// a launch lasts as long as its slowest wave: four lanes then (128^2 rows of
// 12: 7.3 us per Heun step on 4 lanes, 8.5 on 2; from 256^2 on, 2 lanes
// are faster).
// Batching serves configurations whose lane groups are too few to hide
// memory latency with a pipeline (n <= 2^21).  Tuning override
// SPH_EULER_BATCH_LANES = 2 (up to six entries per lane), 4 or 8; 0 turns
// batching off.
int batch_lanes(const sph_ctx* c) {
    int forced = -1;
    if (const char* e = getenv("SPH_EULER_BATCH_LANES")) forced = atoi(e);
    if (forced == 0) return 0;
    if (c->ell_state != 1) return 0;
    if (forced == 2) return (c->ell_S + 1) / 2 <= 6 ? 2 : 0;
    if (forced == 4) return (c->ell_S + 3) / 4 <= 5 ? 4 : 0;
    if (forced == 8) return (c->ell_S + 7) / 8 <= 4 ? 8 : 0;
    if (c->n > (1 << 21)) return 0;
    if ((c->ell_S + 1) / 2 <= 6 && (c->n >= (1 << 15) || (c->ell_S + 3) / 4 > 5)) return 2;
    if ((c->ell_S + 3) / 4 <= 5) return 4;
    return 0;
}

// Lanes per particle: the most (up to 8) that still leave each lane at
// least five row entries.  More lanes put more of a row's gathers in flight
// at once; fewer keep the pipeline over the row deep enough and the lane
// combination cheap (measured on 2-D and 3-D Taylor-Green rows of 12 to 80
// entries).
int lanes_per_particle(const sph_ctx* c) {
    // tuning override: SPH_EULER_LANES = 1, 2, 4 or 8
    if (const char* e = getenv("SPH_EULER_LANES")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8) return v;
    }
    const double avg = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    int L = 1;
    while (L < 8 && avg / (2 * L) >= 5.0) L <<= 1;
    return L;
}

// One stage of the solver SOL (the compressible rows run on the per-particle
// kernel in 2-D only; the caller has checked).
template <int SOL, int STAGE>
void launch(sph_ctx* c, const EulerArgs& ea, const StageIO& io) {
    if (int bl = batch_lanes(c)) {
        bool done;
        if constexpr (SOL == SOL_LINEARISED)
            done = c->dim == 2 ? launch_batch<2, SOL, STAGE>(c, ea, io, bl) : launch_batch<3, SOL, STAGE>(c, ea, io, bl);
        else
            done = launch_batch<2, SOL, STAGE>(c, ea, io, bl);
        if (done) return;
    }
    int L = lanes_per_particle(c);
    if (c->dim == 2) {
        if (L == 1) launch_l<2, SOL, STAGE, 1>(c, ea, io);
        else if (L == 2) launch_l<2, SOL, STAGE, 2>(c, ea, io);
        else if (L == 4) launch_l<2, SOL, STAGE, 4>(c, ea, io);
        else launch_l<2, SOL, STAGE, 8>(c, ea, io);
    } else if constexpr (SOL == SOL_LINEARISED) {
        if (L == 1) launch_l<3, SOL, STAGE, 1>(c, ea, io);
        else if (L == 2) launch_l<3, SOL, STAGE, 2>(c, ea, io);
        else if (L == 4) launch_l<3, SOL, STAGE, 4>(c, ea, io);
        else launch_l<3, SOL, STAGE, 8>(c, ea, io);
    }
}

// 3-D records path: used when the records and the row entries fit the
// 32-bit gathers (n < 2^26 particles, fewer than 2^30 row entries), unless
// the tuning override SPH_EULER_GEO=split selects the separate geometry
// arrays of the generic kernel.
bool use_rec3(const sph_ctx* c) {
    if (c->dim != 3) return false;
    const char* e = getenv("SPH_EULER_GEO");
    if (e && strcmp(e, "split") == 0) return false;
    if ((uint64_t)c->n >= (1ull << 26)) return false;
    const uint64_t entries = c->ell_state == 1 ? (uint64_t)c->ell_S * (uint64_t)c->n : (uint64_t)c->nnz;
    return entries < (1ull << 30);
}

struct Stage3 {
    const float4* R;
    float4* Rout;
    const float4* U;
    const float4* U0;
    float4* Uout;
    float* dr;
    float* dm;
};

template <int STAGE, int L, int M>
void launch3_m(sph_ctx* c, const EulerArgs& ea, const Stage3& io) {
    const dim3 grid(grid_for(c->n, BLK / L));
    if (c->ell_state == 1)
        hipLaunchKernelGGL((k_euler3<STAGE, L, true, M>), grid, dim3(BLK), 0, c->stream, c->n, ea, nullptr,
                           c->colE.as<int32_t>(), c->ell_S, io.R, io.Rout, io.U, io.U0, io.Uout,
                           c->sorted.as<float4>(), io.dr, io.dm);
    else
        hipLaunchKernelGGL((k_euler3<STAGE, L, false, M>), grid, dim3(BLK), 0, c->stream, c->n, ea,
                           c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), 0, io.R, io.Rout, io.U, io.U0, io.Uout,
                           c->sorted.as<float4>(), io.dr, io.dm);
}

// Pairs per chunk: for fixed-stride rows the M in {6, 8, 10, 12, 16} whose
// chunks cover a lane's ceil(S / L) entries with the fewest padding pairs
// (the larger on a tie); CSR rows take chunks of 8.
template <int STAGE, int L>
void launch3_l(sph_ctx* c, const EulerArgs& ea, const Stage3& io) {
    if (c->ell_state != 1) {
        launch3_m<STAGE, L, 8>(c, ea, io);
        return;
    }
    const int mu = (c->ell_S + L - 1) / L;
    const int cand[5] = {16, 12, 10, 8, 6};
    int best = 16, cost = 1 << 30;
    for (int M : cand) {
        const int k = (mu + M - 1) / M * M;
        if (k < cost) cost = k, best = M;
    }
    if (best == 16) launch3_m<STAGE, L, 16>(c, ea, io);
    else if (best == 12) launch3_m<STAGE, L, 12>(c, ea, io);
    else if (best == 10) launch3_m<STAGE, L, 10>(c, ea, io);
    else if (best == 8) launch3_m<STAGE, L, 8>(c, ea, io);
    else launch3_m<STAGE, L, 6>(c, ea, io);
}

// Lanes per particle of the 3-D records kernel: 4 from 16 row entries on
// (measured on the 200^3 Taylor-Green rows, ms per launch for 1, 2, 4, 8
// lanes: 32 entries 1.59, 1.37, 1.34, 1.83; 80 entries 3.81, 3.22, 3.03,
// 3.30), 2 from 6, else 1; tuning override SPH_EULER_LANES.
int lanes3(const sph_ctx* c) {
    if (const char* e = getenv("SPH_EULER_LANES")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8) return v;
    }
    const double avg = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    return avg >= 16.0 ? 4 : (avg >= 6.0 ? 2 : 1);
}


template <int STAGE, int M, int HC, int NT>
void launch3w_h(sph_ctx* c, const EulerArgs& ea, const Stage3& io) {
    const auto& w = c->win3;
    hipLaunchKernelGGL((k_euler3w<STAGE, M, HC, NT>), dim3(grid_for(c->n, NT / 4)), dim3(NT), 0, c->stream,
                       c->n, ea, w.col.as<uint16_t>(), w.Sp, w.off.as<int32_t>(), w.list.as<int32_t>(), io.R,
                       io.Rout, io.U, io.U0, io.Uout, c->sorted.as<float4>(), io.dr, io.dm);
}

// LDS planes for the longest window: 512, 768 or 1024 records (32, 48 or
// 64 KB per workgroup).
template <int STAGE, int M, int NT>
void launch3w_m(sph_ctx* c, const EulerArgs& ea, const Stage3& io) {
    const int32_t mx = c->win3.max;
    if constexpr (NT == 256) {
        if (mx <= 512) {
            launch3w_h<STAGE, M, 512, NT>(c, ea, io);
            return;
        }
    }
    if (mx <= 768) launch3w_h<STAGE, M, 768, NT>(c, ea, io);
    else launch3w_h<STAGE, M, 1024, NT>(c, ea, io);
}

template <int STAGE, int NT>
void launch3w_t(sph_ctx* c, const EulerArgs& ea, const Stage3& io) {
    const int M = c->win3.M;
    if (M == 12) launch3w_m<STAGE, 12, NT>(c, ea, io);
    else if (M == 10) launch3w_m<STAGE, 10, NT>(c, ea, io);
    else if (M == 8) launch3w_m<STAGE, 8, NT>(c, ea, io);
    else launch3w_m<STAGE, 6, NT>(c, ea, io);
}

// Workgroup size of the window kernels (four lanes per particle): 512
// threads, blocks of 128 slots (measured on the 200^3 Taylor-Green rows, ms
// per launch for 256 / 512 threads: 1.20 / 1.13 at 1.6h, 2.25 / 1.76 at 2h;
// blocks of 256 slots need windows beyond 1024 records); tuning override
// SPH_EULER_WINDOW_THREADS = 256 or 512.
int window_threads() {
    if (const char* e = getenv("SPH_EULER_WINDOW_THREADS")) {
        const int v = atoi(e);
        if (v == 256 || v == 512) return v;
    }
    return 512;
}

// Whether the stage kernels read the neighbour records from LDS windows
// (built on first use): fixed-stride rows with four lanes per particle.
int prepare_windows(sph_ctx* c, bool* use) {
    *use = false;
    if (c->ell_state != 1 || lanes3(c) != 4) return SPH_OK;
    if (const char* e = getenv("SPH_EULER_WINDOW"))
        if (strcmp(e, "0") == 0) return SPH_OK;
    const int r = sph_windows_prepare(c, c->win3, 4, window_threads() / 4);
    if (r) return r;
    *use = c->win3.state == 1;
    return SPH_OK;
}

template <int STAGE>
void launch3(sph_ctx* c, const EulerArgs& ea, const Stage3& io, bool windows) {
    const int L = lanes3(c);
    if (windows) {
        if (c->win3.P == 64) launch3w_t<STAGE, 256>(c, ea, io);
        else launch3w_t<STAGE, 512>(c, ea, io);
        return;
    }
    if (L == 1) launch3_l<STAGE, 1>(c, ea, io);
    else if (L == 2) launch3_l<STAGE, 2>(c, ea, io);
    else if (L == 4) launch3_l<STAGE, 4>(c, ea, io);
    else launch3_l<STAGE, 8>(c, ea, io);
}

// Pack the caller's state into U and both record sets (64 B per particle
// each).
int pack3(sph_ctx* c, const EulerArgs& ea, const float* drho, const float* mom, float4* U) {
    SPH_HIP(c, c->rec3.ensure((size_t)c->n * 8 * sizeof(float4)));
    float4* Ra = c->rec3.as<float4>();
    hipLaunchKernelGGL(k_pack3, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, ea, c->sorted.as<float4>(),
                       drho, mom, c->geo0.as<float4>(), c->geo1.as<float4>(), c->geo2.as<float2>(), U, Ra,
                       Ra + 4 * (size_t)c->n);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

EulerArgs make_hllc_args(const sph_ctx* c, const sph_hllc_params* p) {
    EulerArgs a{};
    KernelConsts kc = make_kernel_consts(SPH_WENDLAND, c->dim, c->dom.h);
    a.hinv = kc.hinv;
    a.nhh = -0.5f * kc.hinv;
    a.gamma = (float)p->gamma;
    a.ig1 = (float)(1.0 / (p->gamma - 1.0));
    a.gm1 = (float)(p->gamma - 1.0);
    a.eta_h = (float)p->eta;
    a.fh = -kc.cF;
    a.dt = (float)p->dt;
    for (int ax = 0; ax < 3; ++ax) {
        a.L[ax] = c->box.L[ax];
        a.invL[ax] = c->box.periodic[ax] ? (float)(1.0 / c->box.Ld[ax]) : 0.f;
        a.lo[ax] = c->box.lo[ax];
    }
    a.margin = (float)(c->rc * 1.001);
    return a;
}

int check_hllc(sph_ctx* c, const sph_hllc_params* p, const char* who) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound || !c->geo_valid)
        return sph_fail(c, SPH_ERR_STATE, "%s: needs a bound configuration and a cached correction", who);
    if (c->dim != 2) return sph_fail(c, SPH_ERR_ARG, "%s: 2-D contexts only", who);
    if (c->dom.kernel != SPH_WENDLAND) return sph_fail(c, SPH_ERR_ARG, "%s: Wendland kernel only", who);
    if (!p) return sph_fail(c, SPH_ERR_ARG, "%s: params NULL", who);
    if (!(p->gamma > 1.0)) return sph_fail(c, SPH_ERR_ARG, "%s: gamma must be > 1", who);
    if (!(p->eta >= 0.0)) return sph_fail(c, SPH_ERR_ARG, "%s: eta must be >= 0", who);
    if (c->n >= (1 << 28))
        return sph_fail(c, SPH_ERR_ARG, "%s: %d particles exceed the 2^28 limit of the gathers", who, c->n);
    return SPH_OK;
}

int pack_hllc(sph_ctx* c, float gm1, const float* rho, const float* mom, const float* E, float4* U, float4* P) {
    hipLaunchKernelGGL(k_pack_hllc, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n, gm1,
                       c->sorted.as<float4>(), rho, mom, E, U, P);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
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
    c->euler_path = SPH_PATH_NONE;
    if (c->n == 0) return SPH_OK;
    if (!drho || !mom || !drho_dt || !dmom_dt) return sph_fail(c, SPH_ERR_ARG, "sph_euler_rhs: NULL array");
    SPH_HIP(c, c->ua.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->ta.ensure((size_t)c->n * sizeof(float4)));
    r = sph_ell_prepare(c);
    if (r) return r;
    EulerArgs ea = make_args(c, p);
    if (use_rec3(c)) {
        bool windows = false;
        r = prepare_windows(c, &windows);
        if (r) return r;
        r = pack3(c, ea, drho, mom, c->ua.as<float4>());
        if (r) return r;
        Stage3 io{c->rec3.as<float4>(), nullptr, nullptr, nullptr, nullptr, drho_dt, dmom_dt};
        launch3<0>(c, ea, io, windows);
        SPH_LAUNCH_CHECK(c);
        c->euler_path = windows ? SPH_PATH_WINDOWS : SPH_PATH_RECORDS;
        return SPH_OK;
    }
    r = pack(c, ea.rho_ref, drho, mom, c->ua.as<float4>(), c->ta.as<float4>());
    if (r) return r;
    StageIO io{c->ua.as<float4>(), c->ta.as<float4>(), nullptr, nullptr, nullptr, drho_dt, dmom_dt};
    launch<SOL_LINEARISED, 0>(c, ea, io);
    SPH_LAUNCH_CHECK(c);
    c->euler_path = SPH_PATH_GENERIC;
    return SPH_OK;
}

int sph_euler_step(sph_ctx* c, const sph_euler_params* p, float* drho, float* mom, int32_t nsteps) {
    int r = check(c, p, "sph_euler_step");
    if (r) return r;
    c->euler_path = SPH_PATH_NONE;
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
    r = sph_ell_prepare(c);
    if (r) return r;
    EulerArgs ea = make_args(c, p);
    if (use_rec3(c)) {
        bool windows = false;
        r = prepare_windows(c, &windows);
        if (r) return r;
        r = pack3(c, ea, drho, mom, U);
        if (r) return r;
        float4* Ra = c->rec3.as<float4>();
        float4* Rb = Ra + 4 * (size_t)c->n;
        // stage 1 gathers Ra, writes (U*, Rb); stage 2 gathers Rb, writes (U, Ra) in place
        Stage3 s1{Ra, Rb, U, nullptr, Us, nullptr, nullptr};
        Stage3 s2{Rb, Ra, Us, U, U, nullptr, nullptr};
        for (int32_t s = 0; s < nsteps; ++s) {
            launch3<1>(c, ea, s1, windows);
            launch3<2>(c, ea, s2, windows);
        }
        c->euler_path = windows ? SPH_PATH_WINDOWS : SPH_PATH_RECORDS;
    } else {
        r = pack(c, ea.rho_ref, drho, mom, U, P);
        if (r) return r;
        // stage 1 gathers P, writes (U*, P*); stage 2 gathers P*, writes (U, P) in place
        StageIO s1{U, P, nullptr, Us, Ps, nullptr, nullptr};
        StageIO s2{Us, Ps, U, U, P, nullptr, nullptr};
        for (int32_t s = 0; s < nsteps; ++s) {
            launch<SOL_LINEARISED, 1>(c, ea, s1);
            launch<SOL_LINEARISED, 2>(c, ea, s2);
        }
        c->euler_path = SPH_PATH_GENERIC;
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

int sph_hllc_rhs(sph_ctx* c, const sph_hllc_params* p, const float* rho, const float* mom, const float* E,
                 float* drho_dt, float* dmom_dt, float* dE_dt) {
    int r = check_hllc(c, p, "sph_hllc_rhs");
    if (r) return r;
    c->euler_path = SPH_PATH_NONE;
    if (c->n == 0) return SPH_OK;
    if (!rho || !mom || !E || !drho_dt || !dmom_dt || !dE_dt)
        return sph_fail(c, SPH_ERR_ARG, "sph_hllc_rhs: NULL array");
    SPH_HIP(c, c->ua.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->ta.ensure((size_t)c->n * sizeof(float4)));
    r = sph_ell_prepare(c);
    if (r) return r;
    EulerArgs ea = make_hllc_args(c, p);
    r = pack_hllc(c, ea.gm1, rho, mom, E, c->ua.as<float4>(), c->ta.as<float4>());
    if (r) return r;
    StageIO io{c->ua.as<float4>(), c->ta.as<float4>(), nullptr, nullptr, nullptr, drho_dt, dmom_dt, dE_dt};
    launch<SOL_HLLC, 0>(c, ea, io);
    SPH_LAUNCH_CHECK(c);
    c->euler_path = SPH_PATH_GENERIC;
    return SPH_OK;
}

int sph_hllc_step(sph_ctx* c, const sph_hllc_params* p, float* rho, float* mom, float* E, int32_t nsteps) {
    int r = check_hllc(c, p, "sph_hllc_step");
    if (r) return r;
    c->euler_path = SPH_PATH_NONE;
    if (nsteps < 0) return sph_fail(c, SPH_ERR_ARG, "sph_hllc_step: nsteps < 0");
    if (!(p->dt > 0.0)) return sph_fail(c, SPH_ERR_ARG, "sph_hllc_step: dt must be > 0");
    if (c->n == 0 || nsteps == 0) return SPH_OK;
    if (!rho || !mom || !E) return sph_fail(c, SPH_ERR_ARG, "sph_hllc_step: NULL array");
    SPH_HIP(c, c->ua.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->ub.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->ta.ensure((size_t)c->n * sizeof(float4)));
    SPH_HIP(c, c->tb.ensure((size_t)c->n * sizeof(float4)));
    float4* U = c->ua.as<float4>();
    float4* Us = c->ub.as<float4>();
    float4* P = c->ta.as<float4>();
    float4* Ps = c->tb.as<float4>();
    r = sph_ell_prepare(c);
    if (r) return r;
    EulerArgs ea = make_hllc_args(c, p);
    r = pack_hllc(c, ea.gm1, rho, mom, E, U, P);
    if (r) return r;
    // stage 1 gathers P, writes (U*, P*); stage 2 gathers P*, writes (U, P) in place
    StageIO s1{U, P, nullptr, Us, Ps, nullptr, nullptr, nullptr};
    StageIO s2{Us, Ps, U, U, P, nullptr, nullptr, nullptr};
    for (int32_t s = 0; s < nsteps; ++s) {
        launch<SOL_HLLC, 1>(c, ea, s1);
        launch<SOL_HLLC, 2>(c, ea, s2);
    }
    SPH_LAUNCH_CHECK(c);
    c->euler_path = SPH_PATH_GENERIC;
    hipLaunchKernelGGL(k_unpack_hllc, dim3(grid_for(c->n, BLK)), dim3(BLK), 0, c->stream, c->n,
                       c->sorted.as<float4>(), U, rho, mom, E);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // extern "C"
