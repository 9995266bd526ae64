/*
 * sph_oracle.c -- TEST INFRASTRUCTURE ONLY (not part of the product path).
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the data-parallel
 * hot path of truncated-Wendland SPH as described in
 *   Wang, Zhang, Haidn & Hu, "An efficient truncation scheme for Eulerian and
 *   total Lagrangian SPH methods", arXiv:2405.05155.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the HIP library: every formula is written out again here from
 * the paper, in FP64, with per-particle sums taken in ascending neighbour
 * order.
 *
 * Conventions (the readings of the paper this file follows):
 *  - positions are SoA, pos[a*n + i] for axis a; tensors are row-major
 *    T[i*d*d + a*d + b];
 *  - r_ij = r_i - r_j, with the minimum-image rule on periodic axes;
 *  - grad W_ij is the gradient with respect to r_i,
 *      grad W_ij = (dW/dr)(|r_ij|) * r_ij / |r_ij|,
 *    the only sign that makes the relaxation force (Eq. 7), the correction
 *    matrix (Eq. 9), the Eulerian system (Eq. 19) and the total Lagrangian
 *    system (Eqs. 31-32) physically consistent.  For coincident particles
 *    (|r_ij| = 0) the unit vector is undefined and grad W_ij is taken as 0;
 *  - the neighbour set of i is {j != i : |r_ij|^2 <= rc^2} with |r_ij|^2
 *    evaluated in FP64 as ((dx*dx + dy*dy) + dz*dz) and rc^2 supplied by the
 *    caller (Eq. 5: W = 0 only for |r| > kappa h, so r = kappa h is inside).
 *
 * Parity pins: every function here is checked by tests/test_oracle_pins.py
 * against closed forms, printed values (Table 1), brute force or invariants;
 * see the header comment of each function for what pins it.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int dim;            /* 1, 2 or 3 */
    int periodic[3];    /* per axis, nonzero = periodic */
    double lo[3];
    double hi[3];
} or_box;

enum { OR_WENDLAND = 0, OR_LAGUERRE_GAUSS = 1 };

/* Number of OpenMP threads the oracle's parallel loops use. */
int or_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Kernels                                                             */
/* ------------------------------------------------------------------ */

/* Wendland C2, Eq. (6), Sec. 2.3.1: W = alpha_d (1 - q/2)^4 (2q + 1),
 * q = r/h, alpha_1 = 3/(4h), alpha_2 = 7/(4 pi h^2), alpha_3 = 21/(16 pi h^3).
 * The support test (q <= kappa) is applied by the neighbour set, so this
 * function evaluates the polynomial for any q in [0, 2]. */
static double wendland_alpha(int dim, double h)
{
    if (dim == 1) return 3.0 / (4.0 * h);
    if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
    return 21.0 / (16.0 * M_PI * h * h * h);
}

/* Laguerre-Gauss, Eq. (8), Sec. 2.3.2, read as
 *   W = (a_d / h^d) (1 - q^2 + q^4/6) exp(-q^2),  q <= 2,
 * with a_1 = 8/(5 sqrt(pi)), a_2 = 3/pi, a_3 = 8/pi^(3/2).  The printed
 * polynomial (1 - q^2/2 + q^4/6) does not integrate to one with the printed
 * a_d; the form above does, in 1, 2 and 3 dimensions. */
static double lg_alpha(int dim, double h)
{
    if (dim == 1) return 8.0 / (5.0 * sqrt(M_PI)) / h;
    if (dim == 2) return 3.0 / M_PI / (h * h);
    return 8.0 / pow(M_PI, 1.5) / (h * h * h);
}

double or_kernel_W(int kernel, int dim, double h, double r)
{
    double q = r / h;
    if (kernel == OR_WENDLAND) {
        double t = 1.0 - 0.5 * q;
        return wendland_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
    }
    return lg_alpha(dim, h) * (1.0 - q * q + q * q * q * q / 6.0) * exp(-q * q);
}

/* dW/dr obtained by differentiating the expressions above term by term
 * (product rule, written out, not simplified). */
double or_kernel_dWdr(int kernel, int dim, double h, double r)
{
    double q = r / h;
    if (kernel == OR_WENDLAND) {
        double t = 1.0 - 0.5 * q;
        /* d/dq [t^4 (2q+1)] = 4 t^3 (-1/2) (2q+1) + t^4 * 2 */
        double dq = 4.0 * t * t * t * (-0.5) * (2.0 * q + 1.0) + t * t * t * t * 2.0;
        return wendland_alpha(dim, h) * dq / h;
    }
    {
        double poly = 1.0 - q * q + q * q * q * q / 6.0;
        double dpoly = -2.0 * q + 4.0 * q * q * q / 6.0;
        double e = exp(-q * q);
        double dq = dpoly * e + poly * (-2.0 * q) * e;
        return lg_alpha(dim, h) * dq / h;
    }
}

void or_kernel_eval(int kernel, int dim, double h, int64_t m, const double* r,
                    double* W, double* dWdr)
{
    for (int64_t k = 0; k < m; ++k) {
        if (W) W[k] = or_kernel_W(kernel, dim, h, r[k]);
        if (dWdr) dWdr[k] = or_kernel_dWdr(kernel, dim, h, r[k]);
    }
}

/* ------------------------------------------------------------------ */
/* Pair geometry                                                       */
/* ------------------------------------------------------------------ */

/* r_ij = r_i - r_j with the minimum image on periodic axes. */
static void pair_vec(const or_box* b, int64_t n, const double* pos, int64_t i, int64_t j, double d[3])
{
    for (int a = 0; a < 3; ++a) d[a] = 0.0;
    for (int a = 0; a < b->dim; ++a) {
        double x = pos[a * n + i] - pos[a * n + j];
        if (b->periodic[a]) {
            double L = b->hi[a] - b->lo[a];
            if (x > 0.5 * L) x -= L;
            else if (x < -0.5 * L) x += L;
        }
        d[a] = x;
    }
}

static double dist2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

/* grad_i W_ij = dW/dr * r_ij / r  (0 when r = 0). Returns r. */
static double grad_w(int kernel, int dim, double h, const double d[3], double g[3])
{
    double r = sqrt(dist2(d));
    g[0] = g[1] = g[2] = 0.0;
    if (r > 0.0) {
        double w1 = or_kernel_dWdr(kernel, dim, h, r);
        for (int a = 0; a < dim; ++a) g[a] = w1 * d[a] / r;
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* Neighbour sets                                                      */
/* ------------------------------------------------------------------ */

/* Brute force over all j for the listed rows (rows == NULL: all n rows).
 * Fills row_ptr[0..m]; writes col only when col != NULL and nnz <= cap.
 * Returns nnz. */
int64_t or_neighbors_brute(const or_box* b, int64_t n, const double* pos, double rc2,
                           int64_t m, const int64_t* rows,
                           int64_t* row_ptr, int32_t* col, int64_t cap)
{
    int64_t* cnt = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        int64_t c = 0;
        double d[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            pair_vec(b, n, pos, i, j, d);
            if (dist2(d) <= rc2) ++c;
        }
        cnt[k] = c;
    }
    row_ptr[0] = 0;
    for (int64_t k = 0; k < m; ++k) row_ptr[k + 1] = row_ptr[k] + cnt[k];
    free(cnt);
    int64_t nnz = row_ptr[m];
    if (col && nnz <= cap) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < m; ++k) {
            int64_t i = rows ? rows[k] : k;
            int64_t p = row_ptr[k];
            double d[3];
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                pair_vec(b, n, pos, i, j, d);
                if (dist2(d) <= rc2) col[p++] = (int32_t)j;
            }
        }
    }
    return nnz;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Uniform-grid neighbour search: cells of edge >= rc on every axis, the
 * 3^dim block of cells around each particle's cell (duplicates removed when
 * an axis has fewer than three cells), then the same test as the brute
 * force, then each row sorted ascending.  Pinned against or_neighbors_brute. */
int64_t or_neighbors_grid(const or_box* b, int64_t n, const double* pos, double rc, double rc2,
                          int64_t m, const int64_t* rows, int64_t* row_ptr, int32_t* col, int64_t cap)
{
    int dim = b->dim;
    int64_t nc[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) {
        double L = b->hi[a] - b->lo[a];
        int64_t c = (int64_t)floor(L / (rc * (1.0 + 1e-9)));
        nc[a] = c < 1 ? 1 : c;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t* cell_of = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* cstart = (int64_t*)calloc((size_t)(ncell + 1), sizeof(int64_t));
    int64_t* members = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* coord = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t cidx = 0;
        for (int a = 2; a >= 0; --a) {
            int64_t c = 0;
            if (a < dim) {
                double L = b->hi[a] - b->lo[a];
                c = (int64_t)floor((pos[a * n + i] - b->lo[a]) / L * (double)nc[a]);
                if (c < 0) c = 0;
                if (c > nc[a] - 1) c = nc[a] - 1;
            }
            coord[i * 3 + a] = c;
            cidx = cidx * nc[a] + c;
        }
        cell_of[i] = cidx;
        cstart[cidx + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    {
        int64_t* fill = (int64_t*)malloc((size_t)(ncell > 0 ? ncell : 1) * sizeof(int64_t));
        memcpy(fill, cstart, (size_t)ncell * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) members[fill[cell_of[i]]++] = i;
        free(fill);
    }

    int64_t* cnt = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int64_t nnz = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            row_ptr[0] = 0;
            for (int64_t k = 0; k < m; ++k) row_ptr[k + 1] = row_ptr[k] + cnt[k];
            nnz = row_ptr[m];
            if (!col || nnz > cap) break;
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < m; ++k) {
            int64_t i = rows ? rows[k] : k;
            int64_t cells[27];
            int ncells = 0;
            int64_t lim[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) lim[a] = 1;
            for (int64_t oz = -lim[2]; oz <= lim[2]; ++oz)
                for (int64_t oy = -lim[1]; oy <= lim[1]; ++oy)
                    for (int64_t ox = -lim[0]; ox <= lim[0]; ++ox) {
                        int64_t off[3] = {ox, oy, oz};
                        int64_t cc[3];
                        int ok = 1;
                        for (int a = 0; a < 3; ++a) {
                            int64_t c = coord[i * 3 + a] + off[a];
                            if (a < dim && b->periodic[a]) {
                                c = ((c % nc[a]) + nc[a]) % nc[a];
                            } else if (c < 0 || c >= nc[a]) {
                                ok = 0;
                            }
                            cc[a] = c;
                        }
                        if (!ok) continue;
                        int64_t cidx = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                        int dup = 0;
                        for (int u = 0; u < ncells; ++u) dup |= (cells[u] == cidx);
                        if (!dup) cells[ncells++] = cidx;
                    }
            int64_t c = 0;
            int64_t p = pass ? row_ptr[k] : 0;
            double d[3];
            for (int u = 0; u < ncells; ++u) {
                for (int64_t s = cstart[cells[u]]; s < cstart[cells[u] + 1]; ++s) {
                    int64_t j = members[s];
                    if (j == i) continue;
                    pair_vec(b, n, pos, i, j, d);
                    if (dist2(d) <= rc2) {
                        if (pass) col[p + c] = (int32_t)j;
                        ++c;
                    }
                }
            }
            if (pass) qsort(col + p, (size_t)c, sizeof(int32_t), cmp_i32);
            else cnt[k] = c;
        }
    }
    free(cnt);
    free(cell_of);
    free(cstart);
    free(members);
    free(coord);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Small dense linear algebra (FP64)                                   */
/* ------------------------------------------------------------------ */

/* Inverse by Gauss-Jordan elimination with partial pivoting. Returns the
 * determinant (product of pivots with the row-swap sign). */
static double invert(int d, const double* A, double* Ainv)
{
    double a[3][6];
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < 2 * d; ++c)
            a[r][c] = c < d ? A[r * d + c] : (c - d == r ? 1.0 : 0.0);
    double det = 1.0;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 2 * d; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
            det = -det;
        }
        double p = a[c][c];
        det *= p;
        if (p == 0.0) return 0.0;
        for (int k = 0; k < 2 * d; ++k) a[c][k] /= p;
        for (int r = 0; r < d; ++r) {
            if (r == c) continue;
            double f = a[r][c];
            for (int k = 0; k < 2 * d; ++k) a[r][k] -= f * a[c][k];
        }
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) Ainv[r * d + c] = a[r][d + c];
    return det;
}

static double det_of(int d, const double* A)
{
    if (d == 1) return A[0];
    if (d == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void matmul(int d, const double* A, const double* B, double* C)
{
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            double s = 0.0;
            for (int k = 0; k < d; ++k) s += A[r * d + k] * B[k * d + c];
            C[r * d + c] = s;
        }
}

/* ------------------------------------------------------------------ */
/* Kernel summation, correction matrix, corrected gradient             */
/* ------------------------------------------------------------------ */

/* SPH approximation of f = 1 (Eq. 1 with f = 1; Table 1):
 *   out_i = sum_{j in N(i) U {i}} W_ij V_j,  self term included.
 * Pinned by Table 1 (lattice row) and the closed-form normalisation. */
void or_kernel_sum(const or_box* b, int64_t n, const double* pos, int kernel, double h,
                   int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                   const double* vol, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double s = 0.0, d[3];
        int self_done = 0;
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            if (!self_done && j > i) { s += or_kernel_W(kernel, b->dim, h, 0.0) * vol[i]; self_done = 1; }
            pair_vec(b, n, pos, i, j, d);
            s += or_kernel_W(kernel, b->dim, h, sqrt(dist2(d))) * vol[j];
        }
        if (!self_done) s += or_kernel_W(kernel, b->dim, h, 0.0) * vol[i];
        out[k] = s;
    }
}

/* Kernel-gradient correction matrix, Eq. (9), Sec. 2.3.2:
 *   M_i = sum_j r_ij (x) grad W_ij V_j,   B_i = -M_i^{-1}.
 * Inverse by Gauss-Jordan with partial pivoting.  When
 * |det M_i| < 1e-10 |tr M_i / d|^d the matrix is taken as degenerate and
 * B_i = I is used (the paper gives no rule; this one is a reading).
 * Writes B[k*d*d ...] and returns the number of degenerate rows.
 * Pinned: B_i = I/m on lattices, linear-field exactness of the corrected
 * gradient on jittered sets. */
int64_t or_correction_B(const or_box* b, int64_t n, const double* pos, int kernel, double h,
                        int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                        const double* vol, double* B)
{
    int dim = b->dim;
    int64_t ndeg = 0;
#pragma omp parallel for schedule(static) reduction(+ : ndeg)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double M[9] = {0}, d[3], g[3];
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            pair_vec(b, n, pos, i, j, d);
            grad_w(kernel, dim, h, d, g);
            for (int r = 0; r < dim; ++r)
                for (int c = 0; c < dim; ++c) M[r * dim + c] += d[r] * g[c] * vol[j];
        }
        double tr = 0.0;
        for (int r = 0; r < dim; ++r) tr += M[r * dim + r];
        double scale = pow(fabs(tr / dim), dim);
        double Minv[9];
        double det = det_of(dim, M);
        double* Bi = B + k * dim * dim;
        if (!(fabs(det) >= 1e-10 * scale) || scale == 0.0) {
            for (int r = 0; r < dim; ++r)
                for (int c = 0; c < dim; ++c) Bi[r * dim + c] = (r == c) ? 1.0 : 0.0;
            ndeg += 1;
            continue;
        }
        invert(dim, M, Minv);
        for (int r = 0; r < dim * dim; ++r) Bi[r] = -Minv[r];
    }
    return ndeg;
}

/* Corrected field gradient (Eq. 1 in its difference form, with the
 * correction of Eq. 9):
 *   grad f_i = B_i sum_j (f_j - f_i) grad W_ij V_j,     out[a*m + k].
 * Pinned: exact for linear fields on any non-degenerate set. */
void or_gradient(const or_box* b, int64_t n, const double* pos, int kernel, double h,
                 int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                 const double* vol, const double* B, const double* f, double* out)
{
    int dim = b->dim;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double s[3] = {0, 0, 0}, d[3], g[3];
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            pair_vec(b, n, pos, i, j, d);
            grad_w(kernel, dim, h, d, g);
            for (int a = 0; a < dim; ++a) s[a] += (f[j] - f[i]) * g[a] * vol[j];
        }
        const double* Bi = B + i * dim * dim;
        for (int a = 0; a < dim; ++a) {
            double t = 0.0;
            for (int c = 0; c < dim; ++c) t += Bi[a * dim + c] * s[c];
            out[a * m + k] = t;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Eulerian weakly-compressible SPH with the linearised Riemann solver */
/* ------------------------------------------------------------------ */

typedef struct {
    double c;       /* artificial sound speed */
    double rho0;    /* EOS reference density: p = c^2 (rho - rho0), Eq. (18) */
    double eta;     /* limiter coefficient of Eq. (27) (15 in the paper) */
    double mu;      /* dynamic viscosity of the added viscous term (0: inviscid) */
    double dt;      /* time step of the Heun integrator */
} or_euler_params;

/* Right-hand side of Eq. (19) for the mass and momentum rows, per unit
 * volume:
 *   d rho_i/dt      = -2 sum_j w_j (rho v)* . gradW'_ij
 *   d (rho v)_i/dt  = -2 sum_j w_j [ (rho v (x) v)* + p* I ] . gradW'_ij
 *                     + 2 mu sum_j w_j c_ij (v_i - v_j) (dW/dr)_ij / r_ij
 * with gradW'_ij = (B_i + B_j)/2 gradW_ij (Eq. 28), the Riemann problem
 * posed along n = r_ji / r (left state i, right state j), the linearised
 * solver with its dissipation limiter (Eqs. 26-27), the interface velocity
 *   v* = u* n + ((v_l + v_r)/2 - (u_l + u_r)/2 n)
 * (the tangential part as in the HLLC state of Eq. 22) and the interface
 * density from the EOS, rho* = rho0 + p* / c^2.  The viscous term is not in
 * the paper (its examples state Re only); it is the SPH pair-sum Laplacian
 * with the normalisation c_ij = (tr B_i + tr B_j) / (2 d).  The pair sum
 * applied to a quadratic field weighs it by the second moment
 * sum_j V_j (dW/dr)/r r_ij (x) r_ij = M_i of the correction matrix (Eq. 9),
 * and -tr M_i / d = 1 / (tr B_i / d) on a lattice; the continuum identity
 * -int r W'(r) dV = d holds only for a kernel that vanishes at the cut-off,
 * so without c_ij a truncated kernel under-weights the Laplacian (by 3.3% at
 * 1.6h in 2-D, in the continuum).  With c_ij the term equals mu lap(v) for
 * quadratic fields on a lattice at any cut-off, and stays antisymmetric in
 * the pair (momentum is conserved).
 * Optional abs-sum scales (sum_j |term_ij| per output component) are
 * returned for the tolerance of the parity tests.
 * Pinned: pairwise conservation, the central-flux special case, uniform
 * state -> zero, and a hand-evaluated single pair. */
void or_euler_rhs(const or_box* b, int64_t n, const double* pos, double h,
                  int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                  const double* vol, const double* B, const or_euler_params* prm,
                  const double* rho, const double* mom,
                  double* drho, double* dmom, double* scale_rho, double* scale_mom)
{
    int dim = b->dim;
    double c = prm->c, c2 = c * c;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double sr = 0.0, sm[3] = {0, 0, 0}, ar = 0.0, am[3] = {0, 0, 0};
        double vi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) vi[a] = mom[a * n + i] / rho[i];
        double pi_ = c2 * (rho[i] - prm->rho0);
        const double* Bi = B + i * dim * dim;
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            double d[3], g[3];
            pair_vec(b, n, pos, i, j, d);
            double r = grad_w(OR_WENDLAND, dim, h, d, g);
            if (r == 0.0) continue;
            const double* Bj = B + j * dim * dim;
            double gc[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a)
                for (int q = 0; q < dim; ++q) gc[a] += 0.5 * (Bi[a * dim + q] + Bj[a * dim + q]) * g[q];
            double nrm[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) nrm[a] = -d[a] / r;
            double vj[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) vj[a] = mom[a * n + j] / rho[j];
            double pj = c2 * (rho[j] - prm->rho0);
            double ul = 0.0, ur = 0.0;
            for (int a = 0; a < dim; ++a) { ul += vi[a] * nrm[a]; ur += vj[a] * nrm[a]; }
            double rhobar = 0.5 * (rho[i] + rho[j]);
            double cbar = c;
            double beta = prm->eta * fmax((ul - ur) / cbar, 0.0);
            if (beta > 1.0) beta = 1.0;
            double ustar = 0.5 * (ul + ur) + 0.5 * beta * beta * (pi_ - pj) / (rhobar * cbar);
            double pstar = 0.5 * (pi_ + pj) + 0.5 * beta * rhobar * cbar * (ul - ur);
            double vstar[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a)
                vstar[a] = ustar * nrm[a] + (0.5 * (vi[a] + vj[a]) - 0.5 * (ul + ur) * nrm[a]);
            double rhostar = prm->rho0 + pstar / c2;
            double vg = 0.0;
            for (int a = 0; a < dim; ++a) vg += vstar[a] * gc[a];
            double tr = -2.0 * vol[j] * rhostar * vg;
            sr += tr;
            ar += fabs(tr);
            double w1 = or_kernel_dWdr(OR_WENDLAND, dim, h, r);
            double trB = 0.0;
            for (int a = 0; a < dim; ++a) trB += Bi[a * dim + a] + Bj[a * dim + a];
            double cij = trB / (2.0 * dim);
            for (int a = 0; a < dim; ++a) {
                double tm = -2.0 * vol[j] * (rhostar * vstar[a] * vg + pstar * gc[a]);
                double tv = 2.0 * prm->mu * cij * vol[j] * (vi[a] - vj[a]) * w1 / r;
                sm[a] += tm + tv;
                am[a] += fabs(tm) + fabs(tv);
            }
        }
        drho[k] = sr;
        for (int a = 0; a < dim; ++a) dmom[a * m + k] = sm[a];
        if (scale_rho) scale_rho[k] = ar;
        if (scale_mom)
            for (int a = 0; a < dim; ++a) scale_mom[a * m + k] = am[a];
    }
}

/* Heun (two-stage, strong-stability-preserving) integration with fixed dt:
 *   U* = U + dt R(U);   U <- (U + U* + dt R(U*)) / 2.
 * The paper names no integrator; this is the reading used for the
 * time-stepping parity.  rho, mom updated in place (full n). */
void or_euler_heun(const or_box* b, int64_t n, const double* pos, double h,
                   const int64_t* row_ptr, const int32_t* col,
                   const double* vol, const double* B, const or_euler_params* prm,
                   double* rho, double* mom, int64_t nsteps)
{
    int dim = b->dim;
    double* r1 = (double*)malloc((size_t)n * sizeof(double));
    double* m1 = (double*)malloc((size_t)n * dim * sizeof(double));
    double* dr = (double*)malloc((size_t)n * sizeof(double));
    double* dm = (double*)malloc((size_t)n * dim * sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        or_euler_rhs(b, n, pos, h, n, NULL, row_ptr, col, vol, B, prm, rho, mom, dr, dm, NULL, NULL);
        for (int64_t i = 0; i < n; ++i) r1[i] = rho[i] + prm->dt * dr[i];
        for (int64_t i = 0; i < n * dim; ++i) m1[i] = mom[i] + prm->dt * dm[i];
        or_euler_rhs(b, n, pos, h, n, NULL, row_ptr, col, vol, B, prm, r1, m1, dr, dm, NULL, NULL);
        for (int64_t i = 0; i < n; ++i) rho[i] = 0.5 * (rho[i] + r1[i] + prm->dt * dr[i]);
        for (int64_t i = 0; i < n * dim; ++i) mom[i] = 0.5 * (mom[i] + m1[i] + prm->dt * dm[i]);
    }
    free(r1); free(m1); free(dr); free(dm);
}

/* ------------------------------------------------------------------ */
/* Eulerian compressible SPH: limited HLLC, energy row, ideal gas      */
/* ------------------------------------------------------------------ */

typedef struct {
    double gamma;   /* ideal gas: p = (gamma - 1) (E - rho |v|^2 / 2), E per unit volume */
    double eta;     /* limiter coefficient of the HLLC limiter (1 in the paper) */
    double dt;      /* time step of the Heun integrator */
} or_hllc_params;

/* Interface state of one pair's Riemann problem along the unit vector nrm
 * (left state l = particle i, right state r = particle j), Sec. 3.1:
 *   wave speeds S_l = u_l - c_l, S_r = u_r + c_r (Eq. 20), c = sqrt(gamma p / rho);
 *   the limited middle state (Eq. 24, beta of Eq. 25)
 *     u* = (rho_l c_l u_l + rho_r c_r u_r) / (rho_l c_l + rho_r c_r)
 *          + beta^2 (p_l - p_r) / (rho_l c_l + rho_r c_r),
 *     p* = (p_l + p_r)/2 + beta/2 [rho_r c_r (u* - u_r) + rho_l c_l (u_l - u*)],
 *     beta = min(eta max((u_l - u_r) / cbar, 0), 1), cbar = (c_l + c_r)/2;
 *   (the printed bracket has a minus between its terms; the plus makes p*
 *   the mean of Eq. (22)'s two expressions p_l + rho_l c_l (u_l - u*) and
 *   p_r + rho_r c_r (u* - u_r), and gives the linearised solver's
 *   (p_l + p_r)/2 + beta rho c (u_l - u_r)/2 for equal impedances; with the
 *   minus a head-on collision would raise no pressure);
 *   the HLLC star states (Eq. 22) with the normal velocities u_K where the
 *   printed formulas show |v_K|:
 *     rho*_K = rho_K (S_K - u_K) / (S_K - u*),
 *     E*_K   = ((S_K - u_K) E_K - p_K u_K + p* u*) / (S_K - u*),
 *     v*     = u* n + ((v_l + v_r)/2 - (u_l + u_r)/2 n).
 * Where the two estimates cross (a pair approaching faster than c_l + c_r)
 * the fan is bracketed by S_l = min(u_l - c_l, u_r - c_r) and
 * S_r = max(u_l + c_l, u_r + c_r) instead (Davis's estimates; mirror
 * symmetric like the printed ones).
 * The interface (the pair's midpoint) does not move: the state there is the
 * left state if S_l >= 0, the right state if S_r <= 0, else the left star
 * state if u* >= 0 and the right star state otherwise.
 * Outputs rhoI, vI[dim], pI, EI.  Pinned: equal states give the state back;
 * a supersonic pair gives the upwind state; with beta = 0 the middle state
 * is the impedance-weighted mean velocity and the mean pressure; the state
 * is the same with l and r swapped and nrm reversed (conservation). */
void or_hllc_interface(int dim, const double* nrm, double gamma, double eta,
                       double rho_l, const double* v_l, double p_l,
                       double rho_r, const double* v_r, double p_r,
                       double* rhoI, double* vI, double* pI, double* EI)
{
    double ul = 0.0, ur = 0.0, kl = 0.0, kr = 0.0;
    for (int a = 0; a < dim; ++a) {
        ul += v_l[a] * nrm[a];
        ur += v_r[a] * nrm[a];
        kl += v_l[a] * v_l[a];
        kr += v_r[a] * v_r[a];
    }
    double El = p_l / (gamma - 1.0) + 0.5 * rho_l * kl;
    double Er = p_r / (gamma - 1.0) + 0.5 * rho_r * kr;
    double cl = sqrt(gamma * p_l / rho_l), cr = sqrt(gamma * p_r / rho_r);
    double Sl = ul - cl, Sr = ur + cr;
    if (Sl > Sr) {  /* approach faster than c_l + c_r: the estimates cross */
        Sl = fmin(ul - cl, ur - cr);
        Sr = fmax(ul + cl, ur + cr);
    }
    if (Sl >= 0.0) {
        *rhoI = rho_l; *pI = p_l; *EI = El;
        for (int a = 0; a < dim; ++a) vI[a] = v_l[a];
        return;
    }
    if (Sr <= 0.0) {
        *rhoI = rho_r; *pI = p_r; *EI = Er;
        for (int a = 0; a < dim; ++a) vI[a] = v_r[a];
        return;
    }
    double zl = rho_l * cl, zr = rho_r * cr;
    double cbar = 0.5 * (cl + cr);
    double beta = eta * fmax((ul - ur) / cbar, 0.0);
    if (beta > 1.0) beta = 1.0;
    double us = (zl * ul + zr * ur) / (zl + zr) + beta * beta * (p_l - p_r) / (zl + zr);
    double ps = 0.5 * (p_l + p_r) + 0.5 * beta * (zr * (us - ur) + zl * (ul - us));
    for (int a = 0; a < dim; ++a) vI[a] = us * nrm[a] + (0.5 * (v_l[a] + v_r[a]) - 0.5 * (ul + ur) * nrm[a]);
    *pI = ps;
    if (us >= 0.0) {
        *rhoI = rho_l * (Sl - ul) / (Sl - us);
        *EI = ((Sl - ul) * El - p_l * ul + ps * us) / (Sl - us);
    } else {
        *rhoI = rho_r * (Sr - ur) / (Sr - us);
        *EI = ((Sr - ur) * Er - p_r * ur + ps * us) / (Sr - us);
    }
}

/* Right-hand side of Eq. (19) with all three rows, per unit volume:
 *   d rho_i/dt     = -2 sum_j w_j rho_I v_I . gradW'_ij
 *   d (rho v)_i/dt = -2 sum_j w_j [ rho_I v_I (v_I . gradW'_ij) + p_I gradW'_ij ]
 *   d E_i/dt       = -2 sum_j w_j (E_I + p_I) v_I . gradW'_ij
 * with gradW'_ij = (B_i + B_j)/2 gradW_ij (Eq. 28) and the interface state
 * of or_hllc_interface along n = r_ji / r.  E is the total energy per unit
 * volume.  Optional abs-sum scales as for the weakly compressible rows. */
void or_hllc_rhs(const or_box* b, int64_t n, const double* pos, double h,
                 int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                 const double* vol, const double* B, const or_hllc_params* prm,
                 const double* rho, const double* mom, const double* E,
                 double* drho, double* dmom, double* dE,
                 double* scale_rho, double* scale_mom, double* scale_E)
{
    int dim = b->dim;
    double gm1 = prm->gamma - 1.0;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double sr = 0.0, sm[3] = {0, 0, 0}, se = 0.0, ar = 0.0, am[3] = {0, 0, 0}, ae = 0.0;
        double vi[3] = {0, 0, 0}, ki = 0.0;
        for (int a = 0; a < dim; ++a) {
            vi[a] = mom[a * n + i] / rho[i];
            ki += vi[a] * vi[a];
        }
        double pi_ = gm1 * (E[i] - 0.5 * rho[i] * ki);
        const double* Bi = B + i * dim * dim;
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            double d[3], g[3];
            pair_vec(b, n, pos, i, j, d);
            double r = grad_w(OR_WENDLAND, dim, h, d, g);
            if (r == 0.0) continue;
            const double* Bj = B + j * dim * dim;
            double gc[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a)
                for (int q = 0; q < dim; ++q) gc[a] += 0.5 * (Bi[a * dim + q] + Bj[a * dim + q]) * g[q];
            double nrm[3] = {0, 0, 0};
            for (int a = 0; a < dim; ++a) nrm[a] = -d[a] / r;
            double vj[3] = {0, 0, 0}, kj = 0.0;
            for (int a = 0; a < dim; ++a) {
                vj[a] = mom[a * n + j] / rho[j];
                kj += vj[a] * vj[a];
            }
            double pj = gm1 * (E[j] - 0.5 * rho[j] * kj);
            double rhoI, vI[3] = {0, 0, 0}, pI, EI;
            or_hllc_interface(dim, nrm, prm->gamma, prm->eta, rho[i], vi, pi_, rho[j], vj, pj,
                              &rhoI, vI, &pI, &EI);
            double vg = 0.0;
            for (int a = 0; a < dim; ++a) vg += vI[a] * gc[a];
            double tr = -2.0 * vol[j] * rhoI * vg;
            double te = -2.0 * vol[j] * (EI + pI) * vg;
            sr += tr; ar += fabs(tr);
            se += te; ae += fabs(te);
            for (int a = 0; a < dim; ++a) {
                double tm = -2.0 * vol[j] * (rhoI * vI[a] * vg + pI * gc[a]);
                sm[a] += tm;
                am[a] += fabs(tm);
            }
        }
        drho[k] = sr;
        dE[k] = se;
        for (int a = 0; a < dim; ++a) dmom[a * m + k] = sm[a];
        if (scale_rho) scale_rho[k] = ar;
        if (scale_E) scale_E[k] = ae;
        if (scale_mom)
            for (int a = 0; a < dim; ++a) scale_mom[a * m + k] = am[a];
    }
}

/* Heun integration of the compressible system (as or_euler_heun); rho,
 * mom, E updated in place (full n). */
void or_hllc_heun(const or_box* b, int64_t n, const double* pos, double h,
                  const int64_t* row_ptr, const int32_t* col,
                  const double* vol, const double* B, const or_hllc_params* prm,
                  double* rho, double* mom, double* E, int64_t nsteps)
{
    int dim = b->dim;
    double* r1 = (double*)malloc((size_t)n * sizeof(double));
    double* m1 = (double*)malloc((size_t)n * dim * sizeof(double));
    double* e1 = (double*)malloc((size_t)n * sizeof(double));
    double* dr = (double*)malloc((size_t)n * sizeof(double));
    double* dm = (double*)malloc((size_t)n * dim * sizeof(double));
    double* de = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        or_hllc_rhs(b, n, pos, h, n, NULL, row_ptr, col, vol, B, prm, rho, mom, E, dr, dm, de, NULL, NULL, NULL);
        for (int64_t i = 0; i < n; ++i) { r1[i] = rho[i] + prm->dt * dr[i]; e1[i] = E[i] + prm->dt * de[i]; }
        for (int64_t i = 0; i < n * dim; ++i) m1[i] = mom[i] + prm->dt * dm[i];
        or_hllc_rhs(b, n, pos, h, n, NULL, row_ptr, col, vol, B, prm, r1, m1, e1, dr, dm, de, NULL, NULL, NULL);
        for (int64_t i = 0; i < n; ++i) {
            rho[i] = 0.5 * (rho[i] + r1[i] + prm->dt * dr[i]);
            E[i] = 0.5 * (E[i] + e1[i] + prm->dt * de[i]);
        }
        for (int64_t i = 0; i < n * dim; ++i) mom[i] = 0.5 * (mom[i] + m1[i] + prm->dt * dm[i]);
    }
    free(r1); free(m1); free(e1); free(dr); free(dm); free(de);
}

/* ------------------------------------------------------------------ */
/* Total Lagrangian SPH                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    double rho0;     /* reference density */
    double E;        /* Young's modulus */
    double nu;       /* Poisson ratio */
    double dt;       /* time step */
    int model;       /* 0: compressible neo-Hookean, 1: St. Venant-Kirchhoff (Eq. 30) */
} or_tlsph_params;

/* First Piola-Kirchhoff stress P = F S.
 *  model 1 (Eq. 30): E = (F^T F - I)/2,  S = lambda tr(E) I + 2 G E.
 *  model 0 (compressible neo-Hookean, the law the plate workload names):
 *          S = G (I - C^{-1}) + lambda ln(J) C^{-1},  C = F^T F, J = det F.
 *  lambda = E nu / ((1+nu)(1-2nu)), G = E / (2 (1+nu)). */
void or_tlsph_stress(int dim, const or_tlsph_params* prm, const double* F, double* P)
{
    double lam = prm->E * prm->nu / ((1.0 + prm->nu) * (1.0 - 2.0 * prm->nu));
    double G = prm->E / (2.0 * (1.0 + prm->nu));
    double Ft[9], C[9], S[9];
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) Ft[r * dim + c] = F[c * dim + r];
    matmul(dim, Ft, F, C);
    if (prm->model == 1) {
        double Eg[9], tr = 0.0;
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) Eg[r * dim + c] = 0.5 * (C[r * dim + c] - (r == c ? 1.0 : 0.0));
        for (int r = 0; r < dim; ++r) tr += Eg[r * dim + r];
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) S[r * dim + c] = (r == c ? lam * tr : 0.0) + 2.0 * G * Eg[r * dim + c];
    } else {
        double Ci[9];
        invert(dim, C, Ci);
        double J = det_of(dim, F);
        double lnJ = log(J);
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c)
                S[r * dim + c] = G * ((r == c ? 1.0 : 0.0) - Ci[r * dim + c]) + lam * lnJ * Ci[r * dim + c];
    }
    matmul(dim, F, S, P);
}

/* Eqs. (31)-(32), Sec. 3.2:
 *   dF_i/dt = [ sum_j V0_j (v_j - v_i) (x) grad0 W_ij ] B0_i
 *   rho0 a_i = sum_j (P_i B0_i^T + P_j B0_j^T) grad0 W_ij V0_j
 * (the dot in Eq. 32 is an outer product; this is the form that is exact
 * for linear velocity fields).  Geometry (pos0, neighbours, B0) is the
 * reference configuration.  acc of rows with fixed[i] != 0 is set to 0.
 * dFdt[k*d*d], acc[a*m + k].  Pinned: linear exactness, conservation,
 * F = I -> a = 0. */
void or_tlsph_rhs(const or_box* b, int64_t n, const double* pos0, double h,
                  int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                  const double* vol0, const double* B0, const or_tlsph_params* prm,
                  const double* vel, const double* F, const int32_t* fixed,
                  double* dFdt, double* acc, double* scale_acc)
{
    int dim = b->dim, dd = dim * dim;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double L[9] = {0}, a[3] = {0, 0, 0}, sa[3] = {0, 0, 0};
        double Pi[9], Ai[9], Bt[9];
        or_tlsph_stress(dim, prm, F + i * dd, Pi);
        for (int r = 0; r < dim; ++r)
            for (int c = 0; c < dim; ++c) Bt[r * dim + c] = B0[i * dd + c * dim + r];
        matmul(dim, Pi, Bt, Ai);
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            double d[3], g[3];
            pair_vec(b, n, pos0, i, j, d);
            grad_w(OR_WENDLAND, dim, h, d, g);
            for (int r = 0; r < dim; ++r)
                for (int c = 0; c < dim; ++c)
                    L[r * dim + c] += vol0[j] * (vel[r * n + j] - vel[r * n + i]) * g[c];
            double Pj[9], Aj[9], Btj[9];
            or_tlsph_stress(dim, prm, F + j * dd, Pj);
            for (int r = 0; r < dim; ++r)
                for (int c = 0; c < dim; ++c) Btj[r * dim + c] = B0[j * dd + c * dim + r];
            matmul(dim, Pj, Btj, Aj);
            for (int r = 0; r < dim; ++r) {
                double t = 0.0, ta = 0.0;
                for (int c = 0; c < dim; ++c) {
                    double e = (Ai[r * dim + c] + Aj[r * dim + c]) * g[c] * vol0[j];
                    t += e;
                    ta += fabs(e);
                }
                a[r] += t;
                sa[r] += ta;
            }
        }
        matmul(dim, L, B0 + i * dd, dFdt + k * dd);
        int fx = fixed ? fixed[i] : 0;
        for (int r = 0; r < dim; ++r) {
            acc[r * m + k] = fx ? 0.0 : a[r] / prm->rho0;
            if (scale_acc) scale_acc[r * m + k] = sa[r] / prm->rho0;
        }
    }
}

/* One kick-drift-kick step with fixed dt (the paper gives no integrator):
 *   v^{1/2} = v + dt/2 a;  x += dt v^{1/2};  F += dt dF/dt(v^{1/2});
 *   a <- a(F);  v = v^{1/2} + dt/2 a.
 * Rows with fixed[i] != 0 keep x, v = 0 and F = I; their a is 0.
 * acc must hold a(F) on entry (from or_tlsph_rhs). All arrays full n. */
void or_tlsph_step(const or_box* b, int64_t n, const double* pos0, double h,
                   const int64_t* row_ptr, const int32_t* col,
                   const double* vol0, const double* B0, const or_tlsph_params* prm,
                   const int32_t* fixed, double* pos, double* vel, double* F, double* acc,
                   int64_t nsteps)
{
    int dim = b->dim, dd = dim * dim;
    double* vh = (double*)malloc((size_t)n * dim * sizeof(double));
    double* dF = (double*)malloc((size_t)n * dd * sizeof(double));
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < dim; ++a) {
                int fx = fixed ? fixed[i] : 0;
                vh[a * n + i] = fx ? 0.0 : vel[a * n + i] + 0.5 * prm->dt * acc[a * n + i];
            }
        for (int64_t i = 0; i < n; ++i) {
            if (fixed && fixed[i]) continue;
            for (int a = 0; a < dim; ++a) pos[a * n + i] += prm->dt * vh[a * n + i];
        }
        or_tlsph_rhs(b, n, pos0, h, n, NULL, row_ptr, col, vol0, B0, prm, vh, F, fixed, dF, acc, NULL);
        for (int64_t i = 0; i < n; ++i) {
            if (fixed && fixed[i]) continue;
            for (int e = 0; e < dd; ++e) F[i * dd + e] += prm->dt * dF[i * dd + e];
        }
        /* a(F_new): the dF output of this call is discarded */
        or_tlsph_rhs(b, n, pos0, h, n, NULL, row_ptr, col, vol0, B0, prm, vh, F, fixed, dF, acc, NULL);
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < dim; ++a) {
                int fx = fixed ? fixed[i] : 0;
                vel[a * n + i] = fx ? 0.0 : vh[a * n + i] + 0.5 * prm->dt * acc[a * n + i];
            }
    }
    free(vh);
    free(dF);
}

/* ------------------------------------------------------------------ */
/* Particle relaxation inside a sphere (Eq. 7): Laguerre-Gauss kernel */
/* (Eq. 8), or Wendland C2 (Eq. 6) at its full support 2h, the two    */
/* relaxed distributions of the error analysis (Sec. 2.3.3)           */
/* ------------------------------------------------------------------ */

typedef struct {
    double p0;        /* background pressure of Eq. (7) */
    double rho;       /* density of Eq. (7) */
    double h;         /* smoothing length; support radius 2h for both kernels */
    double center[3]; /* sphere centre */
    double radius;    /* sphere radius; SDF phi = |r - c| - R */
    double kappa;     /* step: displacement per unit acceleration, in h^2 rho / (2 p0) units */
    double mu;        /* damping factor of the carried displacement (0: none carried) */
    double max_move;  /* cap on |u_i| per iteration, in units of h */
    int kernel;       /* OR_LAGUERRE_GAUSS or OR_WENDLAND */
} or_relax_params;

/* Exterior kernel-gradient integral for a sphere (a reading: the paper's
 * relaxation, Eq. 7, has no boundary term; without one the truncated
 * support at the surface pushes particles out).
 *   t_i = int_{|r - c| > R} grad_i W(r_i - r) dV = T(rho_i) e_i,
 * rho_i = |r_i - c|, e_i = (r_i - c)/rho_i.  In spherical coordinates about
 * r_i only the radial component survives:
 *   T = pi int_{s0}^{2h} (-dW/ds) s^2 (1 - clamp(u0, -1, 1)^2) ds,
 *   u0 = (R^2 - rho^2 - s^2) / (2 rho s),  s0 = |R - rho|
 * (the integrand vanishes for s < s0).  Composite Simpson rule with 2000
 * panels in t = sqrt(s - s0), which resolves the steep rise of the
 * integrand just above s0 for particles close to the surface.
 * Pinned against the half-space limit and a direct 3-D quadrature. */
double or_relax_tail(const or_relax_params* prm, double rho_c)
{
    double h = prm->h, R = prm->radius;
    if (rho_c <= 0.0) return 0.0;
    double s0 = fabs(R - rho_c);
    double s1 = 2.0 * h;
    if (s0 >= s1) return 0.0;
    const int NP = 2000;
    double t1 = sqrt(s1 - s0);
    double ht = t1 / NP, acc = 0.0;
    for (int k = 0; k <= NP; ++k) {
        double t = ht * k;
        double s = s0 + t * t;
        double f = 0.0;
        if (s > 0.0) {
            double u0 = (R * R - rho_c * rho_c - s * s) / (2.0 * rho_c * s);
            if (u0 < -1.0) u0 = -1.0;
            if (u0 > 1.0) u0 = 1.0;
            /* ds = 2 t dt */
            f = -or_kernel_dWdr(prm->kernel, 3, h, s) * s * s * (1.0 - u0 * u0) * 2.0 * t;
        }
        double wgt = (k == 0 || k == NP) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        acc += wgt * f;
    }
    return M_PI * acc * ht / 3.0;
}

/* The same exterior integral in 2-D, for a circle of radius R (the error
 * analysis's geometry, Sec. 2.3.3):
 *   t_i = int_{|r - c| > R} grad_i W(r_i - r) dA = T(rho_i) e_i.
 * In polar coordinates about r_i (theta from e_i) the point r_i + s (cos,
 * sin) lies outside where cos(theta) > u0, and only the radial component
 * -dW/ds cos(theta) survives the angular integral:
 *   T = 2 int_{s0}^{2h} (-dW/ds) s sqrt(1 - clamp(u0, -1, 1)^2) ds
 * with u0 and s0 as in 3-D; the same substitution t = sqrt(s - s0) and
 * Simpson rule.  Pinned against the half-plane limit and a direct 2-D
 * quadrature. */
double or_relax_tail2(const or_relax_params* prm, double rho_c)
{
    double h = prm->h, R = prm->radius;
    if (rho_c <= 0.0) return 0.0;
    double s0 = fabs(R - rho_c);
    double s1 = 2.0 * h;
    if (s0 >= s1) return 0.0;
    const int NP = 2000;
    double t1 = sqrt(s1 - s0);
    double ht = t1 / NP, acc = 0.0;
    for (int k = 0; k <= NP; ++k) {
        double t = ht * k;
        double s = s0 + t * t;
        double f = 0.0;
        if (s > 0.0) {
            double u0 = (R * R - rho_c * rho_c - s * s) / (2.0 * rho_c * s);
            if (u0 < -1.0) u0 = -1.0;
            if (u0 > 1.0) u0 = 1.0;
            f = -or_kernel_dWdr(prm->kernel, 2, h, s) * s * sqrt(1.0 - u0 * u0) * 2.0 * t;
        }
        double wgt = (k == 0 || k == NP) ? 1.0 : ((k & 1) ? 4.0 : 2.0);
        acc += wgt * f;
    }
    return 2.0 * acc * ht / 3.0;
}

/* Residual force of the relaxation, Eq. (7) with the kernel of prm:
 *   g_i = sum_j grad W_ij V_j + T(rho_i) e_i
 * (a_i = -(2 p0 / rho) g_i), the sphere's T in 3-D and the circle's in
 * 2-D.  Neighbours at cutoff 2h, non-periodic.
 * g[a*m + k]. */
void or_relax_g(const or_box* b, int64_t n, const double* pos, const or_relax_params* prm,
                int64_t m, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                const double* vol, double* g, double* scale_g)
{
    int dim = b->dim;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = rows ? rows[k] : k;
        double s[3] = {0, 0, 0}, sa[3] = {0, 0, 0}, d[3], gw[3];
        for (int64_t p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
            int64_t j = col[p];
            pair_vec(b, n, pos, i, j, d);
            grad_w(prm->kernel, dim, prm->h, d, gw);
            for (int a = 0; a < dim; ++a) { s[a] += gw[a] * vol[j]; sa[a] += fabs(gw[a] * vol[j]); }
        }
        double e[3] = {0, 0, 0}, rc = 0.0;
        for (int a = 0; a < dim; ++a) { e[a] = pos[a * n + i] - prm->center[a]; rc += e[a] * e[a]; }
        rc = sqrt(rc);
        double T = dim == 2 ? or_relax_tail2(prm, rc) : or_relax_tail(prm, rc);
        for (int a = 0; a < dim; ++a) {
            double t = rc > 0.0 ? T * e[a] / rc : 0.0;
            g[a * m + k] = s[a] + t;
            if (scale_g) scale_g[a * m + k] = sa[a] + fabs(t);
        }
    }
}

/* One relaxation iteration on the full set (neighbours passed in).
 * Eq. (7) gives the relaxation acceleration a_i = -(2 p0/rho) g_i; the
 * paper gives no integrator.  Reading used here: damped motion with a
 * carried per-iteration displacement u (zero at the start),
 *   s   = min(kappa h^2, h / (32 max_i |g_i|))      (no particle is moved
 *          more than h/32 by one force evaluation)
 *   u_i = mu u_i - s g_i,   |u_i| capped at max_move h,
 *   r_i += u_i,
 * then particles with phi > 0 are projected back onto the surface,
 * r -= phi grad(phi), and their u is zeroed.  With mu = 0 and a large
 * kappa this is the pure normalised step (r += a dt^2/2 with
 * dt = 0.25 sqrt(h / max|a|)).
 * Returns the residue R = sqrt(mean_i |h g_i|^2) of the positions on entry. */
double or_relax_step(const or_box* b, int64_t n, double* pos, double* u, const or_relax_params* prm,
                     const int64_t* row_ptr, const int32_t* col, const double* vol, double* g_out)
{
    int dim = b->dim;
    double h = prm->h;
    double* g = g_out ? g_out : (double*)malloc((size_t)n * dim * sizeof(double));
    or_relax_g(b, n, pos, prm, n, NULL, row_ptr, col, vol, g, NULL);
    double res = 0.0, gmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double g2 = 0.0;
        for (int a = 0; a < dim; ++a) g2 += g[a * n + i] * g[a * n + i];
        res += h * h * g2;
        if (sqrt(g2) > gmax) gmax = sqrt(g2);
    }
    res = sqrt(res / (double)(n > 0 ? n : 1));
    if (gmax > 0.0) {
        double step = prm->kappa * h * h;
        double lim = h / (32.0 * gmax);
        if (lim < step) step = lim;
        double cap = prm->max_move * h;
        for (int64_t i = 0; i < n; ++i) {
            double un = 0.0;
            for (int a = 0; a < dim; ++a) {
                u[a * n + i] = prm->mu * u[a * n + i] - step * g[a * n + i];
                un += u[a * n + i] * u[a * n + i];
            }
            un = sqrt(un);
            if (un > cap)
                for (int a = 0; a < dim; ++a) u[a * n + i] *= cap / un;
            double e[3] = {0, 0, 0}, rc = 0.0;
            for (int a = 0; a < dim; ++a) {
                pos[a * n + i] += u[a * n + i];
                e[a] = pos[a * n + i] - prm->center[a];
                rc += e[a] * e[a];
            }
            rc = sqrt(rc);
            double phi = rc - prm->radius;
            if (phi > 0.0 && rc > 0.0) {
                for (int a = 0; a < dim; ++a) {
                    pos[a * n + i] -= phi * e[a] / rc;
                    u[a * n + i] = 0.0;
                }
            }
        }
    }
    if (!g_out) free(g);
    return res;
}
