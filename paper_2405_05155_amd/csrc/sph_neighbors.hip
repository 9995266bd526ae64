// sph_neighbors.hip -- binding a particle configuration: a uniform cell grid
// with Morton-ordered cell keys (counting sort by key, members of a cell in
// ascending caller index), and the exact neighbour sets
// N(i) = {j != i : |r_ij|^2 <= (kappa h)^2} stored
//   - in cell-sorted order with sorted-slot column indices (the layout every
//     pair loop of the library runs on: neighbours of a block of slots lie in
//     a compact region of the sorted arrays), found one wave per particle
//     with ballot compaction, and
//   - on the first export, in caller order with caller indices, each row
//     ascending (the exported CSR; a wave-level bitonic sort per row).
//
// Neighbour decision.  The compact support of Eq. (5) keeps r = kappa h.  The
// squared distance is evaluated in FP64 from the FP32 coordinates with the
// minimum image on periodic axes, as ((dx*dx + dy*dy) + dz*dz) with
// explicitly rounded operations (no contraction), and compared with
// (kappa h)^2 computed once on the host in FP64.  For coordinates that are
// multiples of a power of two (quantised inputs) every step is exact, so the
// set is defined independently of the evaluation order.
#include "sph_internal.h"

#include <climits>
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

// One wave per sorted slot s: the candidates of its 3^dim cell block are
// numbered in traversal order (cells in (z, y, x) order, members in cell
// order) and tested 64 at a time, one per lane, with the exact FP64 rule;
// the hits of each batch are compacted with a wave ballot (a lane's entry is
// the row length so far plus the number of lower lanes that hit), so the
// row comes out in traversal order.  PASS 0: the row length (per slot and
// per caller index).  PASS 1: the sorted row (sorted-slot indices).
constexpr int WPB = BLK / 64;  // waves per block

template <int DIM, int PASS>
__global__ void __launch_bounds__(BLK) k_neigh(int32_t n, BoxArgs b, double rc2, const int32_t* __restrict__ cell_start,
                                               const float4* __restrict__ sorted, int32_t* __restrict__ cnt_s,
                                               int32_t* __restrict__ cnt_u, const int64_t* __restrict__ rp_s,
                                               int32_t* __restrict__ col_s) {
    constexpr int NC = DIM == 2 ? 9 : 27;
    const int lane = (int)(threadIdx.x & 63);
    const int32_t s = (int32_t)blockIdx.x * WPB + (int32_t)(threadIdx.x >> 6);
    if (s >= n) return;  // the whole wave
    const float4 p = sorted[s];
    // lane k < NC: cell k of the block and its slot range
    int32_t c0 = 0, cn = 0;
    if (lane < NC) {
        const int cx = cell_coord(p.x, b.lo[0], b.inv_cell[0], b.nc[0]);
        const int cy = cell_coord(p.y, b.lo[1], b.inv_cell[1], b.nc[1]);
        const int cz = DIM == 3 ? cell_coord(p.z, b.lo[2], b.inv_cell[2], b.nc[2]) : 0;
        int x = cx + lane % 3 - 1, y = cy + (lane / 3) % 3 - 1, z = DIM == 3 ? cz + lane / 9 - 1 : 0;
        bool ok = true;
        if (b.periodic[0]) x = x < 0 ? x + b.nc[0] : (x >= b.nc[0] ? x - b.nc[0] : x);
        else ok = ok && x >= 0 && x < b.nc[0];
        if (b.periodic[1]) y = y < 0 ? y + b.nc[1] : (y >= b.nc[1] ? y - b.nc[1] : y);
        else ok = ok && y >= 0 && y < b.nc[1];
        if (DIM == 3) {
            if (b.periodic[2]) z = z < 0 ? z + b.nc[2] : (z >= b.nc[2] ? z - b.nc[2] : z);
            else ok = ok && z >= 0 && z < b.nc[2];
        }
        if (ok) {
            const int32_t key = cell_key(b, x, y, z);
            c0 = cell_start[key];
            cn = cell_start[key + 1] - c0;
        }
    }
    // exclusive prefix of the cell sizes over lanes 0..NC-1 (NC < 32)
    int32_t inc = cn;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int32_t v = __shfl_up(inc, d, 64);
        if (lane >= d) inc += v;
    }
    const int32_t exc = inc - cn;
    const int32_t total = __shfl(inc, NC - 1, 64);
    const int64_t bs = PASS ? rp_s[s] : 0;
    int32_t count = 0;
    for (int32_t base = 0; base < total; base += 64) {
        const int32_t cidx = base + lane;
        // the candidate's cell: the last k < NC whose block starts at or before it
        int k = 0;
#pragma unroll
        for (int step = 16; step > 0; step >>= 1) {
            const int mid = k + step;
            const int32_t v = __shfl(exc, mid < NC ? mid : NC - 1, 64);
            if (mid < NC && v <= cidx) k = mid;
        }
        const int32_t t = __shfl(c0, k, 64) + (cidx - __shfl(exc, k, 64));
        bool in = false;
        if (cidx < total && t != s) in = is_neighbour<DIM>(p, sorted[t], b, rc2);
        const uint64_t m = __ballot(in);
        if (PASS && in) col_s[bs + count + __popcll(m & ((1ull << lane) - 1ull))] = t;
        count += (int32_t)__popcll(m);
    }
    if (!PASS && lane == 0) {
        cnt_s[s] = count;
        cnt_u[__float_as_int(p.w)] = count;
    }
}

// Ascending sort of 64 R values held R per lane (element r * 64 + lane) by a
// bitonic network: partners 64 apart or more sit in the same lane, closer
// partners in lane ^ j.
template <int R>
__device__ __forceinline__ void wave_sort(int32_t (&x)[R], int lane) {
    constexpr int E = 64 * R;
#pragma unroll
    for (int k = 2; k <= E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int rj = j / 64;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r & rj) continue;
                    const bool asc = ((r * 64 + lane) & k) == 0;
                    const int32_t lo = min(x[r], x[r ^ rj]), hi = max(x[r], x[r ^ rj]);
                    x[r] = asc ? lo : hi;
                    x[r ^ rj] = asc ? hi : lo;
                }
            } else {
                const bool lower = (lane & j) == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int32_t o = __shfl_xor(x[r], j, 64);
                    const bool asc = ((r * 64 + lane) & k) == 0;
                    x[r] = (lower == asc) ? min(x[r], o) : max(x[r], o);
                }
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void export_row(int lane, int32_t len, const int32_t* __restrict__ src,
                                           const float4* __restrict__ sorted, int32_t* __restrict__ dst) {
    int32_t x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        x[r] = e < len ? __float_as_int(sorted[src[e]].w) : INT32_MAX;
    }
    wave_sort<R>(x, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        if (e < len) dst[e] = x[r];
    }
}

// The exported CSR: one wave per sorted slot writes its row in caller
// indices, ascending, at the caller row.  Rows of more than 256 entries
// (very dense configurations) are sorted by lane 0.
__global__ void __launch_bounds__(BLK) k_export_rows(int32_t n, const float4* __restrict__ sorted,
                                                     const int64_t* __restrict__ rp_s, const int32_t* __restrict__ col_s,
                                                     const int64_t* __restrict__ rp_u, int32_t* __restrict__ col_u) {
    const int lane = (int)(threadIdx.x & 63);
    const int32_t s = (int32_t)blockIdx.x * WPB + (int32_t)(threadIdx.x >> 6);
    if (s >= n) return;
    const int64_t k0 = rp_s[s];
    const int32_t len = (int32_t)(rp_s[s + 1] - k0);
    const int32_t* src = col_s + k0;
    int32_t* dst = col_u + rp_u[__float_as_int(sorted[s].w)];
    if (len <= 64) export_row<1>(lane, len, src, sorted, dst);
    else if (len <= 128) export_row<2>(lane, len, src, sorted, dst);
    else if (len <= 256) export_row<4>(lane, len, src, sorted, dst);
    else if (lane == 0) {
        for (int32_t a = 0; a < len; ++a) {
            const int32_t v = __float_as_int(sorted[src[a]].w);
            int32_t q = a - 1;
            while (q >= 0 && dst[q] > v) {
                dst[q + 1] = dst[q];
                --q;
            }
            dst[q + 1] = v;
        }
    }
}

// Largest row length: a grid-stride maximum per thread, a block maximum,
// then one atomic per block.
__global__ void k_row_max(int32_t n, const int32_t* __restrict__ cnt, int32_t* out) {
    __shared__ int32_t wmax[BLK / 64];
    int32_t v = 0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v = max(v, cnt[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLK / 64; ++w) v = max(v, wmax[w]);
        atomicMax(out, v);
    }
}

// colE[k n + i] = entry k of sorted row i (k < row length), else i
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
    const unsigned gmax = grid_for(n, BLK) < 1024u ? grid_for(n, BLK) : 1024u;
    hipLaunchKernelGGL(k_row_max, dim3(gmax), dim3(BLK), 0, c->stream, n, c->cnt_s.as<int32_t>(),
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
    return sph_bin_cells_grid(c, dom, n, pos, 1, false);
}

int sph_bin_cells_grid(sph_ctx* c, const sph_domain* dom, int32_t n, const float* pos, int div, bool linear) {
    if (!c) return SPH_ERR_ARG;
    c->bound = false;
    c->geo_valid = false;
    ++c->geo_gen;
    c->ell_state = 0;
    c->win3.state = 0;
    c->wtl.state = 0;
    c->export_valid = false;
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
    BoxArgs b = make_box_args(*dom, rc, div, linear);
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
    const unsigned gw = (unsigned)((n + WPB - 1) / WPB);  // one wave per slot
    if (n > 0) {
        if (c->dim == 2)
            hipLaunchKernelGGL((k_neigh<2, 0>), dim3(gw), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->cnt_s.as<int32_t>(), cnt_u,
                               nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_neigh<3, 0>), dim3(gw), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), c->cnt_s.as<int32_t>(), cnt_u,
                               nullptr, nullptr);
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
    SPH_HIP(c, c->col_s.ensure((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    if (n > 0 && nnz > 0) {
        if (c->dim == 2)
            hipLaunchKernelGGL((k_neigh<2, 1>), dim3(gw), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), nullptr, nullptr,
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>());
        else
            hipLaunchKernelGGL((k_neigh<3, 1>), dim3(gw), dim3(BLK), 0, c->stream, n, b, c->rc2,
                               c->cell_start.as<int32_t>(), c->sorted.as<float4>(), nullptr, nullptr,
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>());
        SPH_LAUNCH_CHECK(c);
    }
    c->export_valid = false;
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
    if (!c->export_valid && c->n > 0 && c->nnz > 0) {
        // the caller-order rows, built on the first export
        SPH_HIP(c, c->col.ensure((size_t)c->nnz * sizeof(int32_t)));
        hipLaunchKernelGGL(k_export_rows, dim3((unsigned)((c->n + WPB - 1) / WPB)), dim3(BLK), 0, c->stream, c->n,
                           c->sorted.as<float4>(), c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(),
                           c->row_ptr.as<int64_t>(), c->col.as<int32_t>());
        SPH_LAUNCH_CHECK(c);
    }
    c->export_valid = true;
    SPH_HIP(c, hipMemcpyAsync(row_ptr, c->row_ptr.as<int64_t>(), (size_t)(c->n + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, c->stream));
    if (c->nnz > 0)
        SPH_HIP(c, hipMemcpyAsync(col, c->col.as<int32_t>(), (size_t)c->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                  c->stream));
    return SPH_OK;
}

}  // extern "C"
