// sph_ctx.hip -- context lifetime, error reporting, kernel constants and the
// exclusive scans used to turn per-cell / per-row counts into offsets.
#include "sph_internal.h"

int sph_fail(sph_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

KernelConsts make_kernel_consts(int type, int dim, double h) {
    KernelConsts k{};
    k.type = type;
    k.hinv = (float)(1.0 / h);
    if (type == SPH_WENDLAND) {
        // Eq. (6): alpha_2 = 7/(4 pi h^2), alpha_3 = 21/(16 pi h^3)
        double a = dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
        k.cW = (float)a;
        // d/dr [a (1-q/2)^4 (2q+1)] = -5 a q (1-q/2)^3 / h  ->  divided by r = q h
        k.cF = (float)(-5.0 * a / (h * h));
    } else {
        // Eq. (8) read with (1 - q^2 + q^4/6): a_2 = 3/pi, a_3 = 8/pi^{3/2}, times h^-d
        double a = dim == 2 ? 3.0 / M_PI / (h * h) : 8.0 / std::pow(M_PI, 1.5) / (h * h * h);
        k.cW = (float)a;
        // d/dq [(1 - q^2 + q^4/6) e^{-q^2}] = -(q/3) e^{-q^2} (12 - 8 q^2 + q^4)
        k.cF = (float)(-a / (3.0 * h * h));
    }
    return k;
}

BoxArgs make_box_args(const sph_domain& d, double rc, int div, bool linear) {
    BoxArgs b{};
    b.dim = d.dim;
    for (int a = 0; a < 3; ++a) {
        if (a < d.dim) {
            double L = d.hi[a] - d.lo[a];
            long long nc = (long long)std::floor(L / (rc / div * (1.0 + 1e-3)));
            if (nc < 1) nc = 1;
            b.lo[a] = (float)d.lo[a];
            b.L[a] = (float)L;
            b.halfL[a] = (float)(0.5 * L);
            b.nc[a] = (int)nc;
            b.inv_cell[a] = (float)((double)nc / L);
            b.periodic[a] = d.periodic[a] ? 1 : 0;
            b.Ld[a] = L;
            b.halfLd[a] = 0.5 * L;
        } else {
            b.lo[a] = 0.f;
            b.L[a] = 1.f;
            b.halfL[a] = 0.5f;
            b.nc[a] = 1;
            b.inv_cell[a] = 0.f;
            b.periodic[a] = 0;
            b.Ld[a] = 1.0;
            b.halfLd[a] = 0.5;
        }
    }
    // Morton keys when the power-of-two key space stays small
    int m = 1;
    for (int a = 0; a < d.dim; ++a)
        while (m < b.nc[a]) m <<= 1;
    double slots = 1.0;
    for (int a = 0; a < d.dim; ++a) slots *= m;
    b.morton = (!linear && slots <= (double)(1 << 27) && m <= (d.dim == 2 ? 65536 : 1024)) ? 1 : 0;
    return b;
}

int64_t cell_slots(const BoxArgs& b) {
    if (!b.morton) return (int64_t)b.nc[0] * b.nc[1] * b.nc[2];
    int64_t m = 1;
    for (int a = 0; a < b.dim; ++a)
        while (m < b.nc[a]) m <<= 1;
    int64_t s = 1;
    for (int a = 0; a < b.dim; ++a) s *= m;
    return s;
}

extern "C" {

int sph_ctx_create(sph_ctx** out, int dim, void* hip_stream) {
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    if (dim != 2 && dim != 3) return SPH_ERR_ARG;
    sph_ctx* c = new sph_ctx();
    c->dim = dim;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return SPH_ERR_HIP;
    }
    sph_mlp_noalloc_setup(c->device);
    *out = c;
    return SPH_OK;
}

void sph_ctx_destroy(sph_ctx* c) {
    if (!c) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->pos4,        &c->cell_of,      &c->slot,           &c->cell_start,  &c->sorted,
                      &c->cnt,         &c->row_ptr,      &c->col,            &c->cnt_s,       &c->rp_s,
                      &c->col_s,       &c->scan_tmp,     &c->counter,        &c->geo0,        &c->geo1,
                      &c->geo2,        &c->ua,           &c->ub,             &c->ta,          &c->tb,
                      &c->tc,          &c->tail,         &c->svol,           &c->sfield,      &c->partials,
                      &c->relax_scalars, &c->colE, &c->fa, &c->fb, &c->fc, &c->pa, &c->sorted_tmp, &c->rec3,
                      &c->win3.len, &c->win3.off, &c->win3.list, &c->win3.col,
                      &c->wtl.len,  &c->wtl.off,  &c->wtl.list,  &c->wtl.col};
    for (DevBuf* b : bufs) b->release();
    (void)hipSetDevice(prev);
    delete c;
}

const char* sph_last_error(const sph_ctx* c) { return c ? c->err : "null context"; }

int sph_set_stream(sph_ctx* c, void* s) {
    if (!c) return SPH_ERR_ARG;
    c->stream = (hipStream_t)s;
    return SPH_OK;
}

int sph_euler_path(const sph_ctx* c) { return c ? c->euler_path : -1; }

int sph_tlsph_path(const sph_ctx* c) { return c ? c->tlsph_path : -1; }

}  // extern "C"

// ------------------------------------------------------------------ scans
// Three-phase exclusive scan: per-block scan with block totals, a single
// block scanning the totals, then the per-block offset added back.
namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <class Tout>
__device__ Tout block_exclusive_scan(Tout v, Tout* lds, Tout* total) {
    // Hillis-Steele over the block in LDS (SCAN_BLOCK entries)
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        Tout add = t >= off ? lds[t - off] : (Tout)0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    Tout incl = lds[t];
    *total = lds[SCAN_BLOCK - 1];
    __syncthreads();
    return incl - v;
}

template <class Tout>
__global__ void k_scan_tiles(const int32_t* __restrict__ in, Tout* __restrict__ out, Tout* __restrict__ sums,
                             int64_t n) {
    __shared__ Tout lds[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    Tout vals[SCAN_ITEMS];
    Tout run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        Tout v = i < n ? (Tout)in[i] : (Tout)0;
        vals[k] = run;
        run += v;
    }
    Tout total;
    Tout off = block_exclusive_scan<Tout>(run, lds, &total);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = vals[k] + off;
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class Tout>
__global__ void k_scan_sums(Tout* __restrict__ sums, int64_t nb, Tout* __restrict__ total_out) {
    __shared__ Tout lds[SCAN_BLOCK];
    Tout carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_BLOCK) {
        int64_t i = base + threadIdx.x;
        Tout v = i < nb ? sums[i] : (Tout)0;
        Tout tot;
        Tout ex = block_exclusive_scan<Tout>(v, lds, &tot);
        if (i < nb) sums[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <class Tout>
__global__ void k_scan_add(Tout* __restrict__ out, const Tout* __restrict__ sums, int64_t n) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    Tout off = sums[blockIdx.x];
    for (int k = threadIdx.x; k < SCAN_TILE; k += SCAN_BLOCK) {
        int64_t i = base + k;
        if (i < n) out[i] += off;
    }
}

template <class Tout>
int scan_impl(sph_ctx* c, const int32_t* in, Tout* out, int64_t n) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    SPH_HIP(c, c->scan_tmp.ensure((size_t)nb * sizeof(Tout)));
    Tout* sums = c->scan_tmp.as<Tout>();
    hipLaunchKernelGGL(k_scan_tiles<Tout>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, c->stream, in, out, sums, n);
    hipLaunchKernelGGL(k_scan_sums<Tout>, dim3(1), dim3(SCAN_BLOCK), 0, c->stream, sums, nb, out + n);
    hipLaunchKernelGGL(k_scan_add<Tout>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, c->stream, out, sums, n);
    SPH_LAUNCH_CHECK(c);
    return SPH_OK;
}

}  // namespace

int sph_scan_i32_to_i32(sph_ctx* c, const int32_t* in, int32_t* out, int64_t n) {
    return scan_impl<int32_t>(c, in, out, n);
}
int sph_scan_i32_to_i64(sph_ctx* c, const int32_t* in, int64_t* out, int64_t n) {
    return scan_impl<int64_t>(c, in, out, n);
}
