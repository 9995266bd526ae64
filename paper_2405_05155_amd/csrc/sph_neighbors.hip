// sph_neighbors.hip -- binding a particle configuration: a uniform cell grid
// with Morton-ordered cell keys (counting sort by key, members of a cell in
// ascending caller index), and the exact neighbour sets
// N(i) = {j != i : |r_ij|^2 <= (kappa h)^2} stored twice:
//   - in cell-sorted order with sorted-slot column indices (the layout every
//     pair loop of the library runs on: neighbours of a block of slots lie in
//     a compact region of the sorted arrays), and
//   - in caller order with caller indices, each row ascending (the exported
//     CSR).
//
// Neighbour decision.  The compact support of Eq. (5) keeps r = kappa h.  The
// squared distance is evaluated in FP64 from the FP32 coordinates with the
// minimum image on periodic axes, as ((dx*dx + dy*dy) + dz*dz) with
// explicitly rounded operations (no contraction), and compared with
// (kappa h)^2 computed once on the host in FP64.  For coordinates that are
// multiples of a power of two (quantised inputs) every step is exact, so the
// set is defined independently of the evaluation order.
#include "sph_internal.h"

#include <cstdlib>

namespace {

constexpr int BLK = 256;

__global__ void k_bin(int32_t n, int dim, const float* __restrict__ pos, BoxArgs b,
                      float4* __restrict__ pos4, int32_t* __restrict__ cell_of,
                      int32_t* __restrict__ slot, int32_t* __restrict__ count) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = pos[i];
    float y = pos[(int64_t)n + i];
    float z = dim == 3 ? pos[2 * (int64_t)n + i] : 0.f;
    pos4[i] = make_float4(x, y, z, 0.f);
    int cx = cell_coord(x, b.lo[0], b.inv_cell[0], b.nc[0]);
    int cy = cell_coord(y, b.lo[1], b.inv_cell[1], b.nc[1]);
    int cz = dim == 3 ? cell_coord(z, b.lo[2], b.inv_cell[2], b.nc[2]) : 0;
    int32_t key = cell_key(b, cx, cy, cz);
    cell_of[i] = key;
    slot[i] = atomicAdd(&count[key], 1);
}

__global__ void k_scatter(int32_t n, const float4* __restrict__ pos4, const int32_t* __restrict__ cell_of,
                          const int32_t* __restrict__ slot, const int32_t* __restrict__ cell_start,
                          float4* __restrict__ sorted) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 p = pos4[i];
    p.w = __int_as_float(i);
    sorted[cell_start[cell_of[i]] + slot[i]] = p;
}

// Members of each cell in ascending caller index (deterministic order):
// slot s of the provisional (atomic) placement goes to cell start + its rank
// among the cell's members.
__global__ void k_rank_cells(int32_t n, const int32_t* __restrict__ cell_of, const int32_t* __restrict__ cell_start,
                             const float4* __restrict__ tmp, float4* __restrict__ sorted) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 p = tmp[s];
    const int32_t i = __float_as_int(p.w);
    const int32_t key = cell_of[i];
    const int32_t c0 = cell_start[key], c1 = cell_start[key + 1];
    int32_t rank = 0;
    for (int32_t t = c0; t < c1; ++t) rank += __float_as_int(tmp[t].w) < i ? 1 : 0;
    sorted[c0 + rank] = p;
}

__device__ __forceinline__ double md_image(double d, double L, double halfL, int periodic) {
    if (periodic) {
        if (d > halfL) d = __dsub_rn(d, L);
        else if (d < -halfL) d = __dadd_rn(d, L);
    }
    return d;
}

// Visit every sorted slot t in the 3^dim block of cells around p; f(t, q).
template <int DIM, class F>
__device__ __forceinline__ void for_each_candidate(const float4& p, const BoxArgs& b,
                                                   const int32_t* __restrict__ cell_start,
                                                   const float4* __restrict__ sorted, F&& f) {
    int cx = cell_coord(p.x, b.lo[0], b.inv_cell[0], b.nc[0]);
    int cy = cell_coord(p.y, b.lo[1], b.inv_cell[1], b.nc[1]);
    int cz = DIM == 3 ? cell_coord(p.z, b.lo[2], b.inv_cell[2], b.nc[2]) : 0;
    const int zr = DIM == 3 ? 1 : 0;
    for (int oz = -zr; oz <= zr; ++oz) {
        int z = cz + oz;
        if (DIM == 3) {
            if (b.periodic[2]) z = z < 0 ? z + b.nc[2] : (z >= b.nc[2] ? z - b.nc[2] : z);
            else if (z < 0 || z >= b.nc[2]) continue;
        }
        for (int oy = -1; oy <= 1; ++oy) {
            int y = cy + oy;
            if (b.periodic[1]) y = y < 0 ? y + b.nc[1] : (y >= b.nc[1] ? y - b.nc[1] : y);
            else if (y < 0 || y >= b.nc[1]) continue;
            for (int ox = -1; ox <= 1; ++ox) {
                int x = cx + ox;
                if (b.periodic[0]) x = x < 0 ? x + b.nc[0] : (x >= b.nc[0] ? x - b.nc[0] : x);
                else if (x < 0 || x >= b.nc[0]) continue;
                int32_t key = cell_key(b, x, y, z);
                int32_t s1 = cell_start[key + 1];
                for (int32_t s = cell_start[key]; s < s1; ++s) f(s, sorted[s]);
            }
        }
    }
}

template <int DIM>
__device__ __forceinline__ bool is_neighbour(const float4& p, const float4& q, const BoxArgs& b, double rc2) {
    double dx = md_image(__dsub_rn((double)p.x, (double)q.x), b.Ld[0], b.halfLd[0], b.periodic[0]);
    double dy = md_image(__dsub_rn((double)p.y, (double)q.y), b.Ld[1], b.halfLd[1], b.periodic[1]);
    double d2 = __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
    if (DIM == 3) {
        double dz = md_image(__dsub_rn((double)p.z, (double)q.z), b.Ld[2], b.halfLd[2], b.periodic[2]);
        d2 = __dadd_rn(d2, __dmul_rn(dz, dz));
    } else {
        d2 = __dadd_rn(d2, 0.0);
    }
    return d2 <= rc2;
}

// One thread per sorted slot.  PASS 0: neighbour count (stored per slot and
// per caller index).  PASS 1: the sorted row (sorted-slot indices, in
// traversal order) and the caller row (caller indices, then sorted).
template <int DIM, int PASS>
__global__ void k_neigh(int32_t n, BoxArgs b, double rc2, const int32_t* __restrict__ cell_start,
                        const float4* __restrict__ sorted, int32_t* __restrict__ cnt_s, int32_t* __restrict__ cnt_u,
                        const int64_t* __restrict__ rp_s, int32_t* __restrict__ col_s,
                        const int64_t* __restrict__ rp_u, int32_t* __restrict__ col_u) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float4 p = sorted[s];
    int32_t i = __float_as_int(p.w);
    int32_t c = 0;
    int64_t bs = PASS ? rp_s[s] : 0;
    int64_t bu = PASS ? rp_u[i] : 0;
    for_each_candidate<DIM>(p, b, cell_start, sorted, [&](int32_t t, const float4& q) {
        if (t != s && is_neighbour<DIM>(p, q, b, rc2)) {
            if (PASS) {
                col_s[bs + c] = t;
                col_u[bu + c] = __float_as_int(q.w);
            }
            ++c;
        }
    });
    if (!PASS) {
        cnt_s[s] = c;
        cnt_u[i] = c;
        return;
    }
    // the caller row ascending (rows are short and arrive cell by cell)
    int32_t* r = col_u + bu;
    for (int32_t a = 1; a < c; ++a) {
        int32_t v = r[a];
        int32_t k = a - 1;
        while (k >= 0 && r[k] > v) {
            r[k + 1] = r[k];
            --k;
        }
        r[k + 1] = v;
    }
}

// Largest row length: a wave-level maximum, then one atomic per wave.
__global__ void k_row_max(int32_t n, const int32_t* __restrict__ cnt, int32_t* out) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t v = i < n ? cnt[i] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

__global__ void k_fill_ell(int32_t n, int32_t S, const int64_t* __restrict__ rp_s, const int32_t* __restrict__ col_s,
                           int32_t* __restrict__ colE) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k0 = rp_s[i];
    const int32_t len = (int32_t)(rp_s[i + 1] - k0);
    for (int32_t k = 0; k < S; ++k) colE[(int64_t)k * n + i] = k < len ? col_s[k0 + k] : i;
}

}  // namespace

int sph_ell_prepare(sph_ctx* c) {
    if (c->ell_state != 0) return SPH_OK;
    const int32_t n = c->n;
    const char* force = getenv("SPH_PAIR_ROWS");  // tuning override: "csr" keeps the CSR rows
    if (n == 0 || c->nnz == 0 || (force && strcmp(force, "csr") == 0)) {
        c->ell_state = -1;
        return SPH_OK;
    }
    SPH_HIP(c, c->counter.ensure(64));
    SPH_HIP(c, hipMemsetAsync(c->counter.p, 0, 4, c->stream));
    hipLaunchKernelGGL(k_row_max, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, c->cnt_s.as<int32_t>(),
                       c->counter.as<int32_t>());
    SPH_LAUNCH_CHECK(c);
    int32_t S = 0;
    SPH_HIP(c, hipMemcpyAsync(&S, c->counter.p, 4, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    // padding may cost at most half the stored entries; entries are
    // addressed through 32-bit byte offsets
    if ((double)S * n > 1.5 * (double)c->nnz + 1024.0 || (double)S * n * sizeof(int32_t) >= 4294967296.0) {
        c->ell_state = -1;
        return SPH_OK;
    }
    SPH_HIP(c, c->colE.ensure((size_t)S * n * sizeof(int32_t)));
    hipLaunchKernelGGL(k_fill_ell, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, S, c->rp_s.as<int64_t>(),
                       c->col_s.as<int32_t>(), c->colE.as<int32_t>());
    SPH_LAUNCH_CHECK(c);
    c->ell_S = S;
    c->ell_state = 1;
    return SPH_OK;
}

// Validate the domain and bin the positions into the cell grid (sorted
// float4 records with the caller index in .w, and cell offsets).  Used by
// sph_build_cells and, every iteration, by the relaxation.
int sph_bin_cells(sph_ctx* c, const sph_domain* dom, int32_t n, const float* pos) {
    if (!c) return SPH_ERR_ARG;
    c->bound = false;
    c->geo_valid = false;
    c->tiles.valid = false;
    c->tiles.failed = false;
    c->ell_state = 0;
    if (!dom) return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: dom is NULL");
    if (dom->dim != c->dim)
        return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: dom->dim %d != context dim %d", dom->dim, c->dim);
    if (!(dom->h > 0.0) || !(dom->kappa > 0.0)) return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: h and kappa must be > 0");
    if (dom->kernel != SPH_WENDLAND && dom->kernel != SPH_LAGUERRE_GAUSS)
        return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: unknown kernel %d", dom->kernel);
    if (n < 0) return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: n < 0");
    if (n > 0 && !pos) return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: pos is NULL");
    double rc = dom->kappa * dom->h;
    for (int a = 0; a < c->dim; ++a) {
        double L = dom->hi[a] - dom->lo[a];
        if (!(L > 0.0)) return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: empty box on axis %d", a);
        if (dom->periodic[a] && L < 3.0 * rc * (1.0 + 1e-3))
            return sph_fail(c, SPH_ERR_ARG,
                            "sph_build_cells: periodic axis %d of length %g is shorter than 3 kappa h (1+1e-3) = %g", a,
                            L, 3.0 * rc * (1.0 + 1e-3));
    }
    BoxArgs b = make_box_args(*dom, rc);
    int64_t ncell = cell_slots(b);
    if (ncell > (int64_t)1 << 30)
        return sph_fail(c, SPH_ERR_ARG, "sph_build_cells: %lld cells exceed the table limit", (long long)ncell);

    c->dom = *dom;
    c->n = n;
    c->rc = rc;
    c->rc2 = rc * rc;
    c->box = b;
    c->ncell = ncell;

    int64_t nn = n > 0 ? n : 1;
    SPH_HIP(c, c->pos4.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->cell_of.ensure(nn * sizeof(int32_t)));
    SPH_HIP(c, c->slot.ensure(nn * sizeof(int32_t)));
    SPH_HIP(c, c->sorted.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->sorted_tmp.ensure(nn * sizeof(float4)));
    SPH_HIP(c, c->cnt.ensure((ncell + 1 > nn ? ncell + 1 : nn) * sizeof(int32_t)));
    SPH_HIP(c, c->cell_start.ensure((ncell + 1) * sizeof(int32_t)));

    int32_t* count = c->cnt.as<int32_t>();
    SPH_HIP(c, hipMemsetAsync(count, 0, (ncell + 1) * sizeof(int32_t), c->stream));
    if (n > 0) {
        hipLaunchKernelGGL(k_bin, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, c->dim, pos, b,
                           c->pos4.as<float4>(), c->cell_of.as<int32_t>(), c->slot.as<int32_t>(), count);
        SPH_LAUNCH_CHECK(c);
    }
    int rcode = sph_scan_i32_to_i32(c, count, c->cell_start.as<int32_t>(), ncell);
    if (rcode) return rcode;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, c->pos4.as<float4>(),
                           c->cell_of.as<int32_t>(), c->slot.as<int32_t>(), c->cell_start.as<int32_t>(),
                           c->sorted_tmp.as<float4>());
        hipLaunchKernelGGL(k_rank_cells, dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n,
                           c->cell_of.as<int32_t>(), c->cell_start.as<int32_t>(), c->sorted_tmp.as<float4>(),
                           c->sorted.as<float4>());
        SPH_LAUNCH_CHECK(c);
    }
    return SPH_OK;
}

extern "C" {

int sph_build_cells(sph_ctx* c, const sph_domain* dom, int32_t n, const float* pos) {
    int rcode = sph_bin_cells(c, dom, n, pos);
    if (rcode) return rcode;
    BoxArgs b = c->box;
    int64_t nn = n > 0 ? n : 1;
    SPH_HIP(c, c->cnt_s.ensure(nn * sizeof(int32_t)));
    SPH_HIP(c, c->rp_s.ensure((nn + 1) * sizeof(int64_t)));
    SPH_HIP(c, c->row_ptr.ensure((nn + 1) * sizeof(int64_t)));
    int32_t* cnt_u = c->cnt.as<int32_t>();  // the cell counts are consumed by now
    if (n > 0) {
        if (c->dim == 2)
            hipLaunchKernelGGL((k_neigh<2, 0>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->cnt_s.as<int32_t>(), cnt_u,
                               nullptr, nullptr, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_neigh<3, 0>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->cnt_s.as<int32_t>(), cnt_u,
                               nullptr, nullptr, nullptr, nullptr);
        SPH_LAUNCH_CHECK(c);
    }
    rcode = sph_scan_i32_to_i64(c, c->cnt_s.as<int32_t>(), c->rp_s.as<int64_t>(), n);
    if (rcode) return rcode;
    rcode = sph_scan_i32_to_i64(c, cnt_u, c->row_ptr.as<int64_t>(), n);
    if (rcode) return rcode;
    int64_t nnz = 0;
    SPH_HIP(c, hipMemcpyAsync(&nnz, c->row_ptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    c->nnz = nnz;
    SPH_HIP(c, c->col.ensure((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    SPH_HIP(c, c->col_s.ensure((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    if (n > 0 && nnz > 0) {
        if (c->dim == 2)
            hipLaunchKernelGGL((k_neigh<2, 1>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), nullptr, nullptr,
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), c->row_ptr.as<int64_t>(),
                               c->col.as<int32_t>());
        else
            hipLaunchKernelGGL((k_neigh<3, 1>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), nullptr, nullptr,
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), c->row_ptr.as<int64_t>(),
                               c->col.as<int32_t>());
        SPH_LAUNCH_CHECK(c);
    }
    c->bound = true;
    return SPH_OK;
}

int sph_neighbors(sph_ctx* c, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz) {
    if (!c) return SPH_ERR_ARG;
    if (!c->bound) return sph_fail(c, SPH_ERR_STATE, "sph_neighbors: no configuration bound (call sph_build_cells)");
    if (nnz) *nnz = c->nnz;
    if (!row_ptr) return sph_fail(c, SPH_ERR_ARG, "sph_neighbors: row_ptr is NULL");
    if (cap < c->nnz)
        return sph_fail(c, SPH_ERR_CAPACITY, "sph_neighbors: capacity %lld < nnz %lld", (long long)cap, (long long)c->nnz);
    if (c->nnz > 0 && !col) return sph_fail(c, SPH_ERR_ARG, "sph_neighbors: col is NULL");
    SPH_HIP(c, hipMemcpyAsync(row_ptr, c->row_ptr.as<int64_t>(), (size_t)(c->n + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, c->stream));
    if (c->nnz > 0)
        SPH_HIP(c, hipMemcpyAsync(col, c->col.as<int32_t>(), (size_t)c->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                  c->stream));
    return SPH_OK;
}

}  // extern "C"
