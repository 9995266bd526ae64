/*
 * sph.h -- C ABI of the MI355X (gfx950) truncated-Wendland SPH hot path.
 *
 * Method: Wang, Zhang, Haidn & Hu, "An efficient truncation scheme for
 * Eulerian and total Lagrangian SPH methods" (arXiv:2405.05155).
 *
 * General conventions
 *  - Every array argument is a DEVICE pointer (hipMalloc'd or a PyTorch CUDA
 *    tensor) owned by the caller, unless its comment says "(host)".
 *  - Positions and vectors are SoA FP32, x[a*n + i] for axis a.  Tensors are
 *    row-major FP32 [n][dim][dim].  Indices are always the caller's
 *    particle order; the library's internal cell order is invisible.
 *  - A context (sph_ctx) is bound to the device that is current when it is
 *    created and to one HIP stream; every call enqueues its kernels on that
 *    stream and returns before they complete, except the calls that return a
 *    host count (they synchronise the stream).  A context is not
 *    thread-safe.  It owns only scratch memory (cell table, neighbour list,
 *    packed per-particle records).
 *  - Every call returns an int status (SPH_OK = 0).  Arguments are checked
 *    on the host before anything is enqueued; on error nothing is enqueued
 *    and sph_last_error() describes the problem.  Asynchronous HIP failures
 *    surface as SPH_ERR_HIP on a later call.
 *  - Kernel-gradient sign: grad W_ij is the gradient with respect to r_i,
 *    dW/dr (r_i - r_j)/|r_i - r_j| (the sign under which Eqs. 7, 9, 19 and
 *    31-32 of the paper are consistent).
 *  - Precision: pair arithmetic is FP32 with compensated (Kahan) per-particle
 *    sums; the correction matrices are inverted in FP64 and the relaxation
 *    residue is reduced in FP64.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

enum {
    SPH_OK = 0,
    SPH_ERR_ARG = -1,       /* invalid argument (message says which) */
    SPH_ERR_CAPACITY = -2,  /* caller buffer too small; the needed size is returned */
    SPH_ERR_HIP = -3,       /* a HIP runtime call failed */
    SPH_ERR_STATE = -5      /* call out of order (e.g. no configuration bound) */
};

enum { SPH_WENDLAND = 0, SPH_LAGUERRE_GAUSS = 1 };

/* Kernels.
 *  SPH_WENDLAND (Eq. 6, Sec. 2.3.1): W = a_d (1 - q/2)^4 (2q + 1), q = r/h,
 *    a_2 = 7/(4 pi h^2), a_3 = 21/(16 pi h^3); support r <= kappa h with
 *    kappa = 2 (standard) or 1.6 (truncated, Sec. 2.3.1), a hard cut with no
 *    renormalisation.
 *  SPH_LAGUERRE_GAUSS (Eq. 8, Sec. 2.3.2): W = a_d h^-d (1 - q^2 + q^4/6)
 *    exp(-q^2), a_2 = 3/pi, a_3 = 8/pi^(3/2), support r <= 2h.  (The
 *    printed polynomial (1 - q^2/2 + q^4/6) does not normalise with the
 *    printed a_d; this form does.)
 */
typedef struct {
    int dim;            /* 2 or 3 */
    int periodic[3];    /* nonzero: periodic axis (minimum image) */
    double lo[3];       /* box; particles must lie in [lo, hi] (periodic: [lo, hi)) */
    double hi[3];
    double h;           /* smoothing length, > 0 */
    double kappa;       /* cut-off factor: neighbours are j != i with |r_ij| <= kappa h */
    int kernel;         /* SPH_WENDLAND or SPH_LAGUERRE_GAUSS */
} sph_domain;

/* Create a context for `dim` = 2 or 3 on the current device, enqueueing on
 * `hip_stream` (a hipStream_t; NULL = the null stream). */
int sph_ctx_create(sph_ctx** out, int dim, void* hip_stream);
void sph_ctx_destroy(sph_ctx* ctx);
/* Message of the last non-OK return of this context (never NULL). */
const char* sph_last_error(const sph_ctx* ctx);
/* Re-bind the context to another stream of the same device. */
int sph_set_stream(sph_ctx* ctx, void* hip_stream);
/* Which pair-loop variant the context's last sph_euler_rhs, sph_euler_step,
 * sph_hllc_rhs or sph_hllc_step call ran (a diagnostic; every variant gives
 * results within the parity bars, the last two bit-identical to each other):
 *  SPH_PATH_NONE     no such call yet, or it had nothing to do;
 *  SPH_PATH_GENERIC  lane groups per particle gathering separate geometry
 *                    and state arrays (2-D, the compressible rows, or
 *                    configurations beyond the 3-D records' limits);
 *  SPH_PATH_RECORDS  3-D: one 64-byte record (geometry, trace of B, 2p and
 *                    velocity) gathered per neighbour;
 *  SPH_PATH_WINDOWS  3-D: as SPH_PATH_RECORDS, the neighbour records read
 *                    from a window of the workgroup's neighbourhood staged in
 *                    LDS (fixed-stride rows whose windows fit).
 * Returns -1 for a NULL context. */
enum { SPH_PATH_NONE = 0, SPH_PATH_GENERIC = 1, SPH_PATH_RECORDS = 2, SPH_PATH_WINDOWS = 3 };
int sph_euler_path(const sph_ctx* ctx);
/* Which variant of the stress-divergence loop (Eq. 31) the context's last
 * sph_tlsph_rhs or sph_tlsph_step call ran: SPH_PATH_GENERIC (neighbour
 * records gathered through the caches) or SPH_PATH_WINDOWS (read from an LDS
 * window of the workgroup's neighbourhood; fixed-stride rows with four lanes
 * per particle whose windows fit).  Results agree to rounding (the sums take
 * the same pairs in the same order, plus zero-separation padding pairs).
 * SPH_PATH_NONE before such a call.  Returns -1 for a NULL context. */
int sph_tlsph_path(const sph_ctx* ctx);

/* ---------------------------------------------------------------- neighbours
 * sph_build_cells: bind a particle configuration.  Bins the n positions
 * (FP32 SoA [dim][n]) into a uniform grid of cells with edge >= kappa h
 * (counting sort by cell, members of each cell in ascending index), then
 * builds the neighbour set N(i) = {j != i : |r_ij|^2 <= (kappa h)^2} of every
 * particle (the compact support of Eq. 5 with r = kappa h inside), the
 * squared distance evaluated in FP64 from the FP32 inputs as
 * ((dx*dx + dy*dy) + dz*dz) with the minimum image on periodic axes and
 * (kappa h)^2 computed once in FP64 on the host.  Stored as CSR in the
 * caller's order with each row ascending.  Synchronises once (to size the
 * list).  Periodic axes need hi - lo >= 3 (kappa h) (1 + 1e-3).
 * The positions are copied: the caller may reuse `pos` afterwards.
 * Invalidates the cached correction geometry. */
int sph_build_cells(sph_ctx* ctx, const sph_domain* dom, int32_t n, const float* pos);

/* Copy the neighbour CSR of the bound configuration: row_ptr int64 [n+1],
 * col int32 [nnz].  *nnz (host) receives the entry count.  If cap < nnz
 * nothing is written and SPH_ERR_CAPACITY is returned. */
int sph_neighbors(sph_ctx* ctx, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz);

/* ---------------------------------------------------------------- kernel sums
 * SPH approximation of f = 1 (Eq. 1 with f = 1; the quantity of Table 1):
 *   out_i = sum_{j in N(i)} W_ij V_j + W(0) V_i      (self term included).
 * vol FP32 [n], out FP32 [n].  Uses the domain's kernel. */
int sph_kernel_sum(sph_ctx* ctx, const float* vol, float* out);

/* Kernel-gradient correction matrix (Eq. 9, Sec. 2.3.2):
 *   M_i = sum_j r_ij (x) grad W_ij V_j   (FP32 Kahan sums),  B_i = -M_i^{-1}
 * inverted in FP64 (adjugate / determinant).  If |det M_i| <
 * 1e-10 |tr M_i / dim|^dim the row is degenerate and B_i = I.
 * B: FP32 [n][dim][dim] (required); B64: FP64 copy (nullable);
 * n_degenerate (host, nullable): count of degenerate rows (synchronises).
 * Also caches (position, V_i, B_i) in the context for sph_gradient,
 * sph_euler_* and sph_tlsph_*. */
int sph_correction_B(sph_ctx* ctx, const float* vol, float* B, double* B64, int32_t* n_degenerate);

/* Cache caller-supplied volumes and matrices instead (e.g. B = I for the
 * uncorrected "without B" variants).  B FP32 [n][dim][dim], assumed symmetric
 * (only the upper triangle is read). */
int sph_set_correction(sph_ctx* ctx, const float* vol, const float* B);

/* Corrected field gradient (Eq. 1 in difference form with Eq. 9):
 *   grad_i = B_i sum_j (f_j - f_i) grad W_ij V_j.
 * f FP32 [n]; grad FP32 [dim][n].  Needs a cached correction. */
int sph_gradient(sph_ctx* ctx, const float* f, float* grad);

/* ---------------------------------------------------------------- Eulerian SPH
 * Weakly-compressible Eulerian SPH, Eq. (19) (mass and momentum rows) with
 * the corrected gradient of Eq. (28), the linearised Riemann solver and its
 * limiter (Eqs. 26-27) posed along n = (r_j - r_i)/r (left state i), the
 * interface velocity v* = u* n + ((v_l+v_r)/2 - (u_l+u_r)/2 n) and density
 * rho* = rho0 + p* / c^2, EOS p = c^2 (rho - rho0) (Eq. 18), plus the viscous
 * term 2 mu sum_j V_j c_ij (v_i - v_j) (dW/dr)/r with c_ij = (tr B_i + tr B_j)
 * / (2 dim), the normalisation that makes the pair-sum Laplacian exact for
 * quadratic fields on a lattice at either cut-off (Wendland kernel only).
 * State: drho = rho - rho_ref (FP32 [n]; storing the deviation keeps FP32
 * resolution for small density changes) and mom = rho v (FP32 [dim][n]). */
typedef struct {
    double c;        /* sound speed */
    double rho0;     /* EOS reference density */
    double rho_ref;  /* state offset: rho = rho_ref + drho */
    double eta;      /* limiter coefficient of Eq. (27); the paper uses 15 */
    double mu;       /* dynamic viscosity (0: inviscid) */
    double dt;       /* time step for sph_euler_step */
} sph_euler_params;

/* Rates per unit volume: drho_dt FP32 [n], dmom_dt FP32 [dim][n]. */
int sph_euler_rhs(sph_ctx* ctx, const sph_euler_params* prm, const float* drho, const float* mom,
                  float* drho_dt, float* dmom_dt);

/* nsteps Heun steps with fixed dt, in place:
 *   U* = U + dt R(U);  U <- (U + U* + dt R(U*)) / 2.
 * The state is packed once into context scratch, advanced there, and
 * unpacked into drho, mom at the end. */
int sph_euler_step(sph_ctx* ctx, const sph_euler_params* prm, float* drho, float* mom, int32_t nsteps);

/* Compressible Eulerian SPH, 2-D: Eq. (19) with all three rows (mass,
 * momentum, total energy) and the corrected gradient of Eq. (28), the HLLC
 * Riemann solver (Eqs. 20-22) with its dissipation limiter (Eqs. 24-25) posed
 * along n = (r_j - r_i)/r (left state i), ideal gas p = (gamma - 1)
 * (E - rho |v|^2 / 2).  The limited middle state (Eq. 24) is
 *   u* = (z_l u_l + z_r u_r + beta^2 (p_l - p_r)) / (z_l + z_r),
 *   p* = (p_l + p_r)/2 + beta/2 (z_r (u* - u_r) + z_l (u_l - u*)),
 * z = rho c, c = sqrt(gamma p / rho), beta = min(eta max((u_l - u_r) /
 * cbar, 0), 1), cbar = (c_l + c_r)/2 (the printed bracket's minus between
 * its terms is read as a plus: p* is then the mean of Eq. (22)'s two
 * expressions).  Wave speeds S_l = u_l - c_l, S_r = u_r + c_r (Eq. 20), or
 * min(u_l - c_l, u_r - c_r) and max(u_l + c_l, u_r + c_r) where those cross.
 * At the fixed interface: the left (right) state if S_l >= 0 (S_r <= 0),
 * else the star state of Eq. (22) on the side of u*'s sign (with the normal
 * velocity u_K where the printed formulas show |v_K|), velocity u* n plus the
 * mean tangential velocity.  Wendland kernel, 2-D contexts only
 * (SPH_ERR_ARG otherwise).  State: rho FP32 [n] (the density itself), mom = rho v FP32 [2][n],
 * E FP32 [n] (total energy per unit volume). */
typedef struct {
    double gamma;    /* ratio of specific heats, > 1 */
    double eta;      /* limiter coefficient; the paper uses 1 */
    double dt;       /* time step for sph_hllc_step */
} sph_hllc_params;

/* Rates per unit volume: drho_dt FP32 [n], dmom_dt FP32 [2][n], dE_dt FP32 [n]. */
int sph_hllc_rhs(sph_ctx* ctx, const sph_hllc_params* prm, const float* rho, const float* mom, const float* E,
                 float* drho_dt, float* dmom_dt, float* dE_dt);

/* nsteps Heun steps with fixed dt, in place (as sph_euler_step). */
int sph_hllc_step(sph_ctx* ctx, const sph_hllc_params* prm, float* rho, float* mom, float* E, int32_t nsteps);

/* ---------------------------------------------------------------- total Lagrangian SPH
 * Sec. 3.2, with the bound configuration as the reference configuration
 * (positions, V0, B0 from the cached correction):
 *   dF_i/dt = [ sum_j V0_j (v_j - v_i) (x) grad0 W_ij ] B0_i          (Eq. 32)
 *   rho0 a_i = sum_j (P_i B0_i^T + P_j B0_j^T) grad0 W_ij V0_j         (Eq. 31)
 * P = F S with S from model 0 (compressible neo-Hookean:
 * S = G (I - C^-1) + lambda ln J C^-1, C = F^T F, J = det F) or model 1
 * (St. Venant-Kirchhoff, Eq. 30).  lambda = E nu/((1+nu)(1-2nu)),
 * G = E/(2(1+nu)).  3-D only. */
typedef struct {
    double rho0;
    double E;
    double nu;
    double dt;       /* for sph_tlsph_step */
    int model;       /* 0 neo-Hookean, 1 St. Venant-Kirchhoff */
} sph_tlsph_params;

/* vel FP32 [3][n], F FP32 [n][3][3], fixed int32 [n] (nullable; rows with
 * fixed[i] != 0 get acc = 0), dF_dt FP32 [n][3][3], acc FP32 [3][n]. */
int sph_tlsph_rhs(sph_ctx* ctx, const sph_tlsph_params* prm, const float* vel, const float* F,
                  const int32_t* fixed, float* dF_dt, float* acc);

/* nsteps kick-drift-kick steps with fixed dt, in place:
 *   v+ = v + dt/2 a;  x += dt v+;  F += dt dF/dt(v+);  a = a(F);  v = v+ + dt/2 a.
 * acc must hold a(F) on entry (sph_tlsph_rhs) and holds it on exit.  Rows
 * with fixed[i] != 0 keep x, v = 0, F and a = 0.  pos FP32 [3][n] (current
 * positions; the reference positions are the bound configuration). */
int sph_tlsph_step(sph_ctx* ctx, const sph_tlsph_params* prm, const int32_t* fixed, float* pos,
                   float* vel, float* F, float* acc, int32_t nsteps);

/* ---------------------------------------------------------------- particle relaxation
 * Particle relaxation (Eq. 7) of particles filling the sphere (3-D
 * contexts) or the circle (2-D contexts; the geometry of the error
 * analysis) |r - center| < radius, with the Laguerre-Gauss kernel of Eq. 8
 * or the Wendland C2 kernel of Eq. 6 at its full support (the two relaxed
 * distributions of the error analysis, Sec. 2.3.3).  The residual force of
 * particle i is
 *   g_i = sum_{j : |r_ij| <= 2h} grad W_ij V_j + T(rho_i) e_i,
 * where the second term is the integral of grad W over the exterior of
 * the sphere (circle) within the support (rho_i = |r_i - c|, e_i = (r_i -
 * c)/rho_i;
 * the paper's relaxation has no boundary term: this one makes a uniform
 * fill up to the surface force-free).  T is tabulated on the host in FP64
 * by Gauss-Legendre quadrature (16385 entries over phi in [-2h, 2h], linear
 * interpolation).  The acceleration is a_i = -(2 p0/rho) g_i (Eq. 7).
 * One iteration (the paper gives no integrator; this is the damped reading):
 *   s = min(kappa h^2, h / (32 max_i |g_i|));
 *   u_i = damping u_i - s g_i,  |u_i| <= max_move h;   r_i += u_i;
 *   particles outside (phi > 0) are projected onto the surface, u_i = 0.
 * The residue of a configuration is R = sqrt(mean_i |h g_i|^2), reduced in
 * FP64 (two-stage, fixed order: deterministic).
 * The domain supplies h and the box of the cell grid (dom->kernel and
 * dom->kappa are ignored: the kernel is prm->kernel, the cut-off 2h).
 * SPH_ERR_ARG for a kernel other than the two. */
typedef struct {
    double p0;          /* background pressure of Eq. (7) */
    double rho;         /* density of Eq. (7) */
    double center[3];   /* sphere (circle) centre; 2-D reads center[0..1] */
    double radius;      /* sphere (circle) radius */
    double kappa;       /* step coefficient (0.1) */
    double damping;     /* carried-displacement factor (0.9) */
    double max_move;    /* cap on |u_i| per iteration in units of h (0.1) */
    int32_t kernel;     /* SPH_LAGUERRE_GAUSS or SPH_WENDLAND (set it: 0 is Wendland) */
} sph_relax_params;

/* niter iterations in place.  pos FP32 [dim][n] (in/out), u FP32 [dim][n]
 * carried displacement (in/out; zero to start), vol FP32 [n].
 * residue: device FP64 scalar (nullable) receiving the residue of the
 * configuration at the start of the last iteration.  The cell grid is
 * rebuilt every iteration.  Synchronises nothing. */
int sph_relax_step(sph_ctx* ctx, const sph_domain* dom, const sph_relax_params* prm, int32_t n, float* pos,
                   float* u, const float* vol, double* residue, int32_t niter);

/* Residual force and residue of a configuration without moving it.
 * g FP32 [dim][n] (nullable), residue device FP64 scalar (nullable). */
int sph_relax_residue(sph_ctx* ctx, const sph_domain* dom, const sph_relax_params* prm, int32_t n,
                      const float* pos, const float* vol, float* g, double* residue);

/* ---------------------------------------------------------------- learned warm start
 * A small network maps the local neighbourhood of a relaxing particle to a
 * displacement (the paper has no learned component; the network, its inputs
 * and its training follow the relaxation workload):
 *   input x (100): offsets (r_j - r_i)/h of the 32 nearest j != i with
 *     |r_ij| <= 2h, ordered by (|r_ij|^2 in FP64, j), zero-padded; then
 *     phi_i/h and grad phi_i = (r_i - c)/|r_i - c| of the sphere;
 *   y (3) = W3 GELU(W2 GELU(W1 x + b1) + b2) + b3, GELU the exact erf form;
 *   the displacement is h y.
 * Parameters are one FP32 array of SPH_MLP_NPARAMS: W1 [128][100], b1 [128],
 * W2 [128][128], b2 [128], W3 [3][128], b3 [3] (row-major, [out][in]).
 * GEMMs run on BF16 matrix cores with FP32 accumulation; weights, layer
 * inputs and the backward GEMM operands are rounded to BF16 (nearest-even).
 * Features are BF16 (uint16_t bit patterns) rows of SPH_MLP_FEAT_STRIDE
 * entries, the last 28 zero. */
#define SPH_MLP_NPARAMS 29827
#define SPH_MLP_FEAT_STRIDE 128

/* Features of the n particles at pos (FP32 [3][n]) inside the sphere of prm
 * (h and the box from dom): feat [n][SPH_MLP_FEAT_STRIDE] BF16. */
int sph_mlp_features(sph_ctx* ctx, const sph_domain* dom, const sph_relax_params* prm, int32_t n,
                     const float* pos, uint16_t* feat);

/* y for n feature rows: out FP32 [n][3]. */
int sph_mlp_forward(sph_ctx* ctx, const float* params, int32_t n, const uint16_t* feat, float* out);

typedef struct {
    double lr;            /* 0: compute the gradient only, no update */
    double beta1, beta2;
    double eps;
    double weight_decay;  /* decoupled, applied to every parameter */
} sph_adamw_params;

/* One training step on a batch: forward, MSE loss against target FP32
 * [batch][3], backward, and (lr > 0) an AdamW update of the FP32 masters
 * params with moments adam_m, adam_v (FP32 [SPH_MLP_NPARAMS], zero before
 * step 1; step counts from 1).  loss: device FP32 scalar (nullable);
 * grad: device FP32 [SPH_MLP_NPARAMS] receiving the gradient (nullable).
 * Batch sums are reduced in a fixed order (deterministic). */
int sph_mlp_train_step(sph_ctx* ctx, const sph_adamw_params* adam, int64_t step, float* params, float* adam_m,
                       float* adam_v, int32_t batch, const uint16_t* feat, const float* target, float* loss,
                       float* grad);

/* sph_mlp_train_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels, arguments and results (bit for bit), with
 * the training pass's per-workgroup partial records kept in a fixed
 * workspace of the library (32.2 MB per GPU, held until the process ends;
 * room for 256 workgroup records) instead of context scratch.  It calls no
 * allocating routine.  Returns SPH_ERR_CAPACITY if the batch would need more
 * workgroup records than the workspace holds (a device with more than 256
 * compute units and batches of more than 256 x 64 samples) and
 * SPH_ERR_STATE if the workspace could not be located on the context's
 * device.  Every call on a GPU shares that GPU's workspace: calls that
 * overlap on one GPU (other streams, other threads) race. */
int sph_mlp_train_step_noalloc(sph_ctx* ctx, const sph_adamw_params* adam, int64_t step, float* params,
                               float* adam_m, float* adam_v, int32_t batch, const uint16_t* feat, const float* target,
                               float* loss, float* grad);

/* One epoch of training steps on rows of a resident training set of nrows
 * rows: step b (b = 0 .. nbatch-1, AdamW step number step0 + b) takes the
 * batch rows[b * batch .. (b + 1) * batch) (int64 indices into feat
 * [nrows][SPH_MLP_FEAT_STRIDE] and target [nrows][3]), gathered inside the
 * training kernel, with the same arithmetic as sph_mlp_train_step on that
 * batch.  An index outside [0, nrows) is clamped to the nearest row.
 * lr must be > 0.  losses: device FP32 [nbatch] receiving each step's loss
 * (nullable). */
int sph_mlp_train_epoch(sph_ctx* ctx, const sph_adamw_params* adam, int64_t step0, float* params, float* adam_m,
                        float* adam_v, int32_t batch, int32_t nbatch, int64_t nrows, const int64_t* rows,
                        const uint16_t* feat, const float* target, float* losses);

/* Training targets of the warm start from two configurations of the same
 * particles: target FP32 [n][3] = (to - from) / h (from, to FP32 [3][n]),
 * the displacement in units of h that the network's output y stands for
 * (the move is r += h y). */
int sph_mlp_targets(sph_ctx* ctx, int32_t n, double h, const float* from, const float* to, float* target);

/* Warm-start move: features of the current positions, y, then r += h y for
 * every particle and the same projection onto the sphere as the relaxation.
 * pos FP32 [3][n] in place. */
int sph_mlp_apply(sph_ctx* ctx, const sph_domain* dom, const sph_relax_params* prm, int32_t n, float* pos,
                  const float* params);

#ifdef __cplusplus
}
#endif

#endif /* SPH_MI355X_H */
