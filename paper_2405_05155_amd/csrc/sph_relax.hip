// sph_relax.hip -- particle relaxation (Eq. 7) of particles filling a
// sphere (3-D) or a circle (2-D, the error analysis's geometry), with the
// Laguerre-Gauss kernel of Eq. 8 or the Wendland C2 kernel of Eq. 6 at its
// full support 2h (the two relaxed distributions of the error analysis,
// Sec. 2.3.3), with the exterior-tail term, an FP64 residue reduction and
// the damped move + surface bound.
//
// Per iteration: re-bin (cells of edge >= h, linear (z, y, x) keys), one
// thread per particle in cell order scans the 5 x 5 x 5 cells (2-D: 5 x 5)
// around its own as contiguous x-runs, a two-stage reduction gives max|g|
// and the FP64 residue, then one thread per particle moves it.
#include "sph_internal.h"

#include <vector>

namespace {

constexpr int BLK = 256;
constexpr int NTAIL = 16385;  // table entries over phi in [-2h, 2h]

// ------------------------------------------------------------------ host: tail table

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
// Legendre polynomial of degree m from the Chebyshev-like initial guesses).
void gauss_legendre(int m, double* x, double* w) {
    for (int i = 0; i < (m + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= m; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = m * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs(z - z1) < 1e-15) break;
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// T(phi), the exterior integral of grad W along e_i, with u0 = (R^2 - rho^2
// - s^2)/(2 rho s), rho = R + phi, and the relaxation's kernel:
//   3-D (sphere): T = pi int_{|phi|}^{2h} (-dW/ds) s^2 (1 - clamp(u0)^2) ds,
//   2-D (circle): T = 2 int_{|phi|}^{2h} (-dW/ds) s sqrt(1 - clamp(u0)^2) ds
// (the exterior arc about r_i at distance s is cos(theta) > u0, and the
// radial component of grad W is -dW/ds cos(theta)).
// Substitution s = s0 + (2h - s0) tau^2 and graded Gauss-Legendre panels in
// tau (dense near tau = 0, where the integrand rises steeply for particles
// just inside the surface).
double tail_integral(int kernel, int dim, double h, double R, double phi) {
    const double rho = R + phi;
    if (rho <= 0.0) return 0.0;
    const double s0 = std::fabs(phi), s1 = 2.0 * h;
    if (s0 >= s1) return 0.0;
    struct GL16 {
        double x[16], w[16];
        GL16() { gauss_legendre(16, x, w); }
    };
    static const GL16 gl;  // thread-safe one-time initialisation
    const double* gx = gl.x;
    const double* gw = gl.w;
    // kernel normalisation a_d h^-d (Eq. 6: 7/(4 pi), 21/(16 pi); Eq. 8: 3/pi, 8/pi^(3/2))
    const double a3 = dim == 2 ? (kernel == SPH_WENDLAND ? 7.0 / (4.0 * M_PI) : 3.0 / M_PI) / (h * h)
                               : (kernel == SPH_WENDLAND ? 21.0 / (16.0 * M_PI) : 8.0 / std::pow(M_PI, 1.5)) / (h * h * h);
    const double edges[] = {0.0, 1.0 / 128, 1.0 / 32, 1.0 / 8, 0.25, 0.5, 0.75, 1.0};
    const double span = s1 - s0;
    double acc = 0.0;
    for (int p = 0; p + 1 < (int)(sizeof(edges) / sizeof(edges[0])); ++p) {
        double a = edges[p], b = edges[p + 1];
        for (int k = 0; k < 16; ++k) {
            double tau = 0.5 * (a + b) + 0.5 * (b - a) * gx[k];
            double s = s0 + span * tau * tau;
            if (s <= 0.0) continue;
            double q = s / h;
            double q2 = q * q;
            double mdw;
            if (kernel == SPH_WENDLAND) {
                // -dW/ds = (a3 / h) 5 q (1 - q/2)^3
                double t = 1.0 - 0.5 * q;
                mdw = a3 / h * 5.0 * q * t * t * t;
            } else {
                // -dW/ds = (a3 / (3 h)) q e^{-q^2} (12 - 8 q^2 + q^4)
                mdw = a3 / (3.0 * h) * q * std::exp(-q2) * (12.0 - 8.0 * q2 + q2 * q2);
            }
            double u0 = (R * R - rho * rho - s * s) / (2.0 * rho * s);
            u0 = u0 < -1.0 ? -1.0 : (u0 > 1.0 ? 1.0 : u0);
            double f = dim == 2 ? mdw * s * std::sqrt(1.0 - u0 * u0) : mdw * s * s * (1.0 - u0 * u0);
            acc += 0.5 * (b - a) * gw[k] * f * 2.0 * span * tau;
        }
    }
    return dim == 2 ? 2.0 * acc : M_PI * acc;
}

int ensure_tail(sph_ctx* c, int kernel, double h, double R) {
    // the table's key: kernel and dimension (tail_kernel = kernel + 4 dim), h, R
    const int key = kernel + 4 * c->dim;
    if (c->ntail == NTAIL && c->tail_kernel == key && c->tail_h == h && c->tail_R == R && c->tail.p) return SPH_OK;
    std::vector<float> tab(NTAIL);
    for (int k = 0; k < NTAIL; ++k) {
        double phi = -2.0 * h + 4.0 * h * k / (NTAIL - 1);
        tab[k] = (float)tail_integral(kernel, c->dim, h, R, phi);
    }
    SPH_HIP(c, c->tail.ensure(NTAIL * sizeof(float)));
    SPH_HIP(c, hipMemcpyAsync(c->tail.p, tab.data(), NTAIL * sizeof(float), hipMemcpyHostToDevice, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));  // the host vector goes out of scope
    c->ntail = NTAIL;
    c->tail_kernel = key;
    c->tail_h = h;
    c->tail_R = R;
    return SPH_OK;
}

// ------------------------------------------------------------------ device

// The relaxation bins on cells RELAX_DIV times finer than the cut-off, with
// linear (z, y, x) keys: a particle's candidates are then the (2 RELAX_DIV +
// 1)^2 contiguous x-runs of 2 RELAX_DIV + 1 cells around it, a block 2.5 cut-offs
// wide instead of the 3 of whole-cut-off cells (about 58% of the candidates).
constexpr int RELAX_DIV = 2;

struct RelaxArgs {
    BoxArgs b;
    int D;           // cells per cut-off (the scan reaches D cells each way)
    float cF;        // (dW/dr)/r: LG cF e^{-q^2} (12 - 8 q^2 + q^4); Wendland cF (1 - q/2)^3
    float hinv;      // 1/h
    float hinv2;     // 1/h^2
    float rc2f;      // (2h)^2 in FP32
    double rc2d;     // (2h)^2 in FP64
    float c[3], R;   // sphere (2-D: circle, c[2] = 0)
    float h, phi_lo, inv_dphi;
    double hh;       // h^2 (FP64, residue)
    float kappa_h2;  // kappa h^2
    float h32;       // h / 32
    float damping, cap;
};

struct RelaxScalars {
    double residue;
    float gmax;
    float step;
    int move;  // 0 when max|g| = 0
};

__device__ __forceinline__ int ccoord(float x, float lo, float inv, int nc) {
    int c = (int)floorf((x - lo) * inv);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

__device__ __forceinline__ double dwrap(double d, double L, double halfL, int periodic) {
    if (periodic) {
        if (d > halfL) d = __dsub_rn(d, L);
        else if (d < -halfL) d = __dadd_rn(d, L);
    }
    return d;
}

// exact neighbour decision (same rule as the neighbour search)
__device__ __forceinline__ bool exact_in(const float4& p, const float4& q, const BoxArgs& b, double rc2) {
    double dx = dwrap(__dsub_rn((double)p.x, (double)q.x), b.Ld[0], b.halfLd[0], b.periodic[0]);
    double dy = dwrap(__dsub_rn((double)p.y, (double)q.y), b.Ld[1], b.halfLd[1], b.periodic[1]);
    double dz = dwrap(__dsub_rn((double)p.z, (double)q.z), b.Ld[2], b.halfLd[2], b.periodic[2]);
    double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    return d2 <= rc2;
}

__device__ __forceinline__ float tail_at(const float* __restrict__ tail, const RelaxArgs& ra, float phi) {
    float x = (phi - ra.phi_lo) * ra.inv_dphi;
    if (!(x > 0.f)) return 0.f;  // phi <= -2h: the support lies inside (also NaN)
    if (x >= (float)(NTAIL - 1)) return tail[NTAIL - 1];
    int k = (int)x;
    float f = x - (float)k;
    return fmaf(f, tail[k + 1] - tail[k], tail[k]);
}

// (dW/dr)/r of the relaxation kernel at squared distance r2.
template <int K>
__device__ __forceinline__ float relax_dwr(float r2, const RelaxArgs& ra) {
    if constexpr (K == SPH_WENDLAND) {
        const float t = 1.f - 0.5f * (sqrtf(r2) * ra.hinv);
        return ra.cF * t * t * t;
    } else {
        const float q2 = r2 * ra.hinv2;
        return ra.cF * __expf(-q2) * (12.f - 8.f * q2 + q2 * q2);
    }
}

// One slot range of candidates of particle s (slot) at p.
template <int K>
__device__ __forceinline__ void relax_range(int32_t t0, int32_t t1, int32_t s, const float4& p, const RelaxArgs& ra,
                                            const float4* __restrict__ rec, Kahan* g) {
    const BoxArgs& b = ra.b;
    for (int32_t t = t0; t < t1; ++t) {
        if (t == s) continue;
        const float4 q = ld32(rec, (uint32_t)t);
        const float d0 = min_image(p.x - q.x, b.L[0], b.halfL[0], b.periodic[0]);
        const float d1 = min_image(p.y - q.y, b.L[1], b.halfL[1], b.periodic[1]);
        const float d2 = min_image(p.z - q.z, b.L[2], b.halfL[2], b.periodic[2]);
        const float r2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        bool in = r2 <= ra.rc2f;
        if (fabsf(r2 - ra.rc2f) <= 1e-5f * ra.rc2f) in = exact_in(p, q, b, ra.rc2d);
        if (!in) continue;
        const float w = relax_dwr<K>(r2, ra) * q.w;
        g[0].add(w * d0);
        g[1].add(w * d1);
        g[2].add(w * d2);
    }
}

// Residual force g_i (caller order) and per-block partials of max|g| and
// sum |h g|^2 (FP64).  One thread per particle in cell order scans the cells
// within D cells of its own (linear keys: for each (z, y) row one contiguous
// slot range, split in two where a periodic x axis wraps); the FP32 distance
// test is redone in FP64 within 1e-5 of the cut-off.  rec holds (x, y, z, V)
// per sorted slot, so a candidate costs one 16-byte load.
template <int K>
__global__ void __launch_bounds__(BLK) k_relax_g(int32_t n, RelaxArgs ra, const int32_t* __restrict__ cell_start,
                                                 const float4* __restrict__ sorted, const float4* __restrict__ rec,
                                                 const float* __restrict__ tail, float4* __restrict__ gout,
                                                 float* __restrict__ part_max, double* __restrict__ part_sum) {
    __shared__ float smax[BLK];
    __shared__ double ssum[BLK];
    const int32_t s = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * BLK + threadIdx.x;
    float gmag = 0.f;
    double gh2 = 0.0;
    if (s < n) {
        const BoxArgs& b = ra.b;
        const float4 p = ld32(rec, (uint32_t)s);
        Kahan g[3];
        g[0].init(); g[1].init(); g[2].init();
        const int cx = ccoord(p.x, b.lo[0], b.inv_cell[0], b.nc[0]);
        const int cy = ccoord(p.y, b.lo[1], b.inv_cell[1], b.nc[1]);
        const int cz = ccoord(p.z, b.lo[2], b.inv_cell[2], b.nc[2]);
        const int D = ra.D, nx = b.nc[0];
        for (int oz = -D; oz <= D; ++oz) {
            int z = cz + oz;
            if (b.periodic[2]) z = z < 0 ? z + b.nc[2] : (z >= b.nc[2] ? z - b.nc[2] : z);
            else if (z < 0 || z >= b.nc[2]) continue;
            for (int oy = -D; oy <= D; ++oy) {
                int y = cy + oy;
                if (b.periodic[1]) y = y < 0 ? y + b.nc[1] : (y >= b.nc[1] ? y - b.nc[1] : y);
                else if (y < 0 || y >= b.nc[1]) continue;
                const int32_t row = (z * b.nc[1] + y) * nx;
                int xa = cx - D, xb = cx + D;
                if (b.periodic[0]) {  // nx >= 2 D + 1: at most one side wraps
                    if (xa < 0) {
                        relax_range<K>(cell_start[row + xa + nx], cell_start[row + nx], s, p, ra, rec, g);
                        xa = 0;
                    } else if (xb >= nx) {
                        relax_range<K>(cell_start[row], cell_start[row + xb - nx + 1], s, p, ra, rec, g);
                        xb = nx - 1;
                    }
                } else {
                    xa = xa < 0 ? 0 : xa;
                    xb = xb > nx - 1 ? nx - 1 : xb;
                }
                relax_range<K>(cell_start[row + xa], cell_start[row + xb + 1], s, p, ra, rec, g);
            }
        }
        // exterior-tail term
        const int32_t i = __float_as_int(sorted[s].w);
        const float ex = p.x - ra.c[0], ey = p.y - ra.c[1], ez = p.z - ra.c[2];
        const float rr = sqrtf(ex * ex + ey * ey + ez * ez);
        const float phi = rr - ra.R;
        if (rr > 0.f) {
            const float T = tail_at(tail, ra, phi) / rr;
            g[0].add(T * ex);
            g[1].add(T * ey);
            g[2].add(T * ez);
        }
        const float gx = g[0].value(), gy = g[1].value(), gz = g[2].value();
        gout[i] = make_float4(gx, gy, gz, 0.f);
        const double g2 = (double)gx * gx + (double)gy * gy + (double)gz * gz;
        gh2 = ra.hh * g2;
        gmag = (float)sqrt(g2);
    }
    smax[threadIdx.x] = gmag;
    ssum[threadIdx.x] = gh2;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_max[blockIdx.x] = smax[0];
        part_sum[blockIdx.x] = ssum[0];
    }
}

// Final reduction (one block, fixed order): residue (FP64), max|g>, step.
__global__ void k_relax_reduce(int32_t nb, int32_t n, RelaxArgs ra, const float* __restrict__ part_max,
                               const double* __restrict__ part_sum, RelaxScalars* __restrict__ out,
                               double* __restrict__ residue) {
    __shared__ float smax[BLK];
    __shared__ double ssum[BLK];
    float m = 0.f;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nb; k += BLK) {
        m = fmaxf(m, part_max[k]);
        acc += part_sum[k];
    }
    smax[threadIdx.x] = m;
    ssum[threadIdx.x] = acc;
    __syncthreads();
    for (int w = BLK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + w]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double res = sqrt(ssum[0] / (double)(n > 0 ? n : 1));
        float gmax = smax[0];
        out->residue = res;
        out->gmax = gmax;
        out->move = gmax > 0.f;
        double lim = gmax > 0.f ? (double)ra.h32 / (double)gmax : 0.0;
        out->step = (float)(lim < (double)ra.kappa_h2 ? lim : (double)ra.kappa_h2);
        if (residue) *residue = res;
    }
}

// u = damping u - step g (capped), r += u, bound to the sphere (circle).
template <int DIM>
__global__ void k_relax_move(int32_t n, RelaxArgs ra, const RelaxScalars* __restrict__ sc,
                             const float4* __restrict__ g, float* __restrict__ pos, float* __restrict__ u) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!sc->move) return;
    float step = sc->step;
    float4 gi = g[i];
    int64_t nn = n;
    float u0 = ra.damping * u[i] - step * gi.x;
    float u1 = ra.damping * u[nn + i] - step * gi.y;
    float u2 = DIM == 3 ? ra.damping * u[2 * nn + i] - step * gi.z : 0.f;
    float un = sqrtf(u0 * u0 + u1 * u1 + u2 * u2);
    if (un > ra.cap) {
        float f = ra.cap / un;
        u0 *= f;
        u1 *= f;
        u2 *= f;
    }
    float x = pos[i] + u0, y = pos[nn + i] + u1, z = DIM == 3 ? pos[2 * nn + i] + u2 : 0.f;
    float ex = x - ra.c[0], ey = y - ra.c[1], ez = z - ra.c[2];
    float rr = sqrtf(ex * ex + ey * ey + ez * ez);
    float phi = rr - ra.R;
    if (phi > 0.f && rr > 0.f) {
        float f = phi / rr;
        x -= f * ex;
        y -= f * ey;
        z -= f * ez;
        u0 = u1 = u2 = 0.f;
    }
    pos[i] = x;
    pos[nn + i] = y;
    u[i] = u0;
    u[nn + i] = u1;
    if (DIM == 3) {
        pos[2 * nn + i] = z;
        u[2 * nn + i] = u2;
    }
}

// (x, y, z, V) per sorted slot
__global__ void k_sorted_rec(int32_t n, const float4* __restrict__ sorted, const float* __restrict__ vol,
                             float4* __restrict__ rec) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 p = sorted[s];
    rec[s] = make_float4(p.x, p.y, p.z, vol[__float_as_int(p.w)]);
}

__global__ void k_unpack_g(int32_t n, int dim, const float4* __restrict__ g4, float* __restrict__ g) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 v = g4[i];
    g[i] = v.x;
    g[(int64_t)n + i] = v.y;
    if (dim == 3) g[2 * (int64_t)n + i] = v.z;
}

int check(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, const void* pos,
          const float* vol, const char* who) {
    if (!c) return SPH_ERR_ARG;

    if (!dom || !p) return sph_fail(c, SPH_ERR_ARG, "%s: NULL domain or params", who);
    if (n < 0) return sph_fail(c, SPH_ERR_ARG, "%s: n < 0", who);
    if (n > 0 && (!pos || !vol)) return sph_fail(c, SPH_ERR_ARG, "%s: NULL array", who);
    if (!(p->radius > 0.0) || !(p->p0 > 0.0) || !(p->rho > 0.0))
        return sph_fail(c, SPH_ERR_ARG, "%s: need radius, p0, rho > 0", who);
    if (!(p->kappa > 0.0) || !(p->damping >= 0.0 && p->damping < 1.0) || !(p->max_move > 0.0))
        return sph_fail(c, SPH_ERR_ARG, "%s: need kappa > 0, 0 <= damping < 1, max_move > 0", who);
    if (p->kernel != SPH_LAGUERRE_GAUSS && p->kernel != SPH_WENDLAND)
        return sph_fail(c, SPH_ERR_ARG, "%s: kernel must be SPH_LAGUERRE_GAUSS or SPH_WENDLAND", who);
    return SPH_OK;
}

RelaxArgs make_args(const sph_ctx* c, const sph_relax_params* p) {
    RelaxArgs ra{};
    double h = c->dom.h;
    ra.b = c->box;
    ra.D = RELAX_DIV;
    KernelConsts kc = make_kernel_consts(p->kernel, c->dim, h);
    ra.cF = kc.cF;
    ra.hinv = kc.hinv;
    ra.hinv2 = (float)(1.0 / (h * h));
    ra.rc2d = c->rc2;
    ra.rc2f = (float)c->rc2;
    for (int a = 0; a < 3; ++a) ra.c[a] = a < c->dim ? (float)p->center[a] : 0.f;
    ra.R = (float)p->radius;
    ra.h = (float)h;
    ra.phi_lo = (float)(-2.0 * h);
    ra.inv_dphi = (float)((NTAIL - 1) / (4.0 * h));
    ra.hh = h * h;
    // the force scale 2 p0 / rho cancels in the normalised step; kappa is in h^2 per unit g
    ra.kappa_h2 = (float)(p->kappa * h * h);
    ra.h32 = (float)(h / 32.0);
    ra.damping = (float)p->damping;
    ra.cap = (float)(p->max_move * h);
    return ra;
}

// bin + g + reduce; leaves g (float4, caller order) in c->ta and the scalars in c->relax_scalars
int relax_eval(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, const float* pos,
               const float* vol, double* residue, RelaxArgs* ra_out) {
    sph_domain d = *dom;
    d.kernel = p->kernel;
    d.kappa = 2.0;
    int r = sph_bin_cells_grid(c, &d, n, pos, RELAX_DIV, true);
    if (r) return r;
    r = ensure_tail(c, p->kernel, d.h, p->radius);
    if (r) return r;
    RelaxArgs ra = make_args(c, p);
    *ra_out = ra;
    int64_t nn = n > 0 ? n : 1;
    int nb = (int)grid_for(nn, BLK);
    SPH_HIP(c, c->svol.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->ta.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->partials.ensure((size_t)nb * (sizeof(float) + sizeof(double)) + 64));
    SPH_HIP(c, c->relax_scalars.ensure(sizeof(RelaxScalars)));
    double* psum = c->partials.as<double>();
    float* pmax = reinterpret_cast<float*>(psum + nb);
    if (n > 0) {
        hipLaunchKernelGGL(k_sorted_rec, dim3(nb), dim3(BLK), 0, c->stream, n, c->sorted.as<float4>(), vol,
                           c->svol.as<float4>());
        if (p->kernel == SPH_WENDLAND)
            hipLaunchKernelGGL(k_relax_g<SPH_WENDLAND>, dim3(nb), dim3(BLK), 0, c->stream, n, ra,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->svol.as<float4>(),
                               c->tail.as<float>(), c->ta.as<float4>(), pmax, psum);
        else
            hipLaunchKernelGGL(k_relax_g<SPH_LAGUERRE_GAUSS>, dim3(nb), dim3(BLK), 0, c->stream, n, ra,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->svol.as<float4>(),
                               c->tail.as<float>(), c->ta.as<float4>(), pmax, psum);
    }
    hipLaunchKernelGGL(k_relax_reduce, dim3(1), dim3(BLK), 0, c->stream, n > 0 ? nb : 0, n, ra, pmax, psum,
                       c->relax_scalars.as<RelaxScalars>(), residue);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // namespace

extern "C" {

int sph_relax_step(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, float* pos, float* u,
                   const float* vol, double* residue, int32_t niter) {
    int r = check(c, dom, p, n, pos, vol, "sph_relax_step");
    if (r) return r;
    if (niter < 0) return sph_fail(c, SPH_ERR_ARG, "sph_relax_step: niter < 0");
    if (n > 0 && !u) return sph_fail(c, SPH_ERR_ARG, "sph_relax_step: u is NULL");
    for (int32_t it = 0; it < niter; ++it) {
        RelaxArgs ra;
        r = relax_eval(c, dom, p, n, pos, vol, it == niter - 1 ? residue : nullptr, &ra);
        if (r) return r;
        if (n > 0) {
            if (c->dim == 2)
                hipLaunchKernelGGL(k_relax_move<2>, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, ra,
                                   c->relax_scalars.as<RelaxScalars>(), c->ta.as<float4>(), pos, u);
            else
                hipLaunchKernelGGL(k_relax_move<3>, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, ra,
                                   c->relax_scalars.as<RelaxScalars>(), c->ta.as<float4>(), pos, u);
            SPH_LAUNCH_CHECK(c);
        }
    }
    return SPH_OK;
}

int sph_relax_residue(sph_ctx* c, const sph_domain* dom, const sph_relax_params* p, int32_t n, const float* pos,
                      const float* vol, float* g, double* residue) {
    int r = check(c, dom, p, n, pos, vol, "sph_relax_residue");
    if (r) return r;
    RelaxArgs ra;
    r = relax_eval(c, dom, p, n, pos, vol, residue, &ra);
    if (r) return r;
    if (g && n > 0) {
        hipLaunchKernelGGL(k_unpack_g, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, c->dim, c->ta.as<float4>(),
                           g);
        SPH_LAUNCH_CHECK(c);
    }
    return SPH_OK;
}

}  // extern "C"
