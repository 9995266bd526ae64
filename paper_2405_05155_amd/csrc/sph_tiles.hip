// sph_tiles.hip -- cell tiles of a fixed configuration for the LDS-staged
// pair loops (the neighbour sets of Eq. (5) are fixed for the Eulerian and
// total-Lagrangian configurations, so the tiles are built once per binding).
//
// A tile is an aligned block of 2^bits consecutive Morton cell keys.  The
// low key bits interleave the axes (x, y[, z], x, ...), so the block is a
// box of cells with power-of-two sides, and its particles are one contiguous
// range of cell-sorted slots.  Since cells are at least the cut-off wide,
// every neighbour of an own particle lies in the box or in its one-cell
// ring; the ring's particles (the halo) are listed per tile, ascending by
// slot, so a workgroup can stage all records its pair loop touches in LDS.
//
// The pair work of a tile is a list of tasks, one per unique neighbour pair
// of its own rows (the fluxes evaluated on it are antisymmetric, so a pair
// of two own particles is evaluated once and written to both rows).
#include "sph_internal.h"

#include <cstdlib>
#include <type_traits>

namespace {

constexpr int BLK = 256;
constexpr int MAX_RING = 512;  // ring cells of the largest tile (8x8x8 cells: 488)

__device__ __forceinline__ uint32_t compact2(uint32_t x) {  // even bits -> 16 bits
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0f0f0f0fu;
    x = (x | (x >> 4)) & 0x00ff00ffu;
    x = (x | (x >> 8)) & 0x0000ffffu;
    return x;
}
__device__ __forceinline__ uint32_t compact3(uint32_t x) {  // every third bit -> 10 bits
    x &= 0x09249249u;
    x = (x | (x >> 2)) & 0x030c30c3u;
    x = (x | (x >> 4)) & 0x0300f00fu;
    x = (x | (x >> 8)) & 0x030000ffu;
    x = (x | (x >> 16)) & 0x000003ffu;
    return x;
}

// Cells per axis of a tile of 2^bits keys: axis a takes key bits a, a + dim, ...
__host__ __device__ __forceinline__ int tile_side(int bits, int dim, int a) {
    if (a >= dim) return 1;
    int nb = bits > a ? (bits - a + dim - 1) / dim : 0;
    return 1 << nb;
}

// First cell and extent (clipped to the grid) of Morton tile T.
__device__ __forceinline__ void tile_box(const BoxArgs& b, int bits, int32_t T, int o[3], int s[3]) {
    uint32_t k0 = (uint32_t)T << bits;
    if (b.dim == 2) {
        o[0] = (int)compact2(k0);
        o[1] = (int)compact2(k0 >> 1);
        o[2] = 0;
    } else {
        o[0] = (int)compact3(k0);
        o[1] = (int)compact3(k0 >> 1);
        o[2] = (int)compact3(k0 >> 2);
    }
    for (int a = 0; a < 3; ++a) {
        int side = tile_side(bits, b.dim, a);
        int lim = b.nc[a] - o[a];
        s[a] = side < lim ? side : lim;
    }
}

__global__ void k_tile_flags(int32_t nT, int bits, const int32_t* __restrict__ cell_start, int32_t* __restrict__ flag) {
    int32_t T = blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= nT) return;
    flag[T] = cell_start[(int64_t)(T + 1) << bits] > cell_start[(int64_t)T << bits] ? 1 : 0;
}

__global__ void k_tile_list(int32_t nT, int bits, const int32_t* __restrict__ flag, const int32_t* __restrict__ tidx,
                            const int32_t* __restrict__ cell_start, int32_t* __restrict__ tlist,
                            int32_t* __restrict__ own_begin, int32_t* __restrict__ own_cnt) {
    int32_t T = blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= nT || !flag[T]) return;
    int32_t t = tidx[T];
    int32_t b0 = cell_start[(int64_t)T << bits];
    tlist[t] = T;
    own_begin[t] = b0;
    own_cnt[t] = cell_start[(int64_t)(T + 1) << bits] - b0;
}

// One workgroup per tile.  The ring cells are collected, ordered by key
// (so their slot ranges ascend), and their offsets in the halo list formed.
// PASS 0 stores the halo count; PASS 1 writes the halo slots.
template <int PASS>
__global__ void __launch_bounds__(BLK) k_tile_ring(int32_t ntile, int bits, BoxArgs b,
                                                   const int32_t* __restrict__ cell_start,
                                                   const int32_t* __restrict__ tlist, int32_t* __restrict__ halo_cnt,
                                                   const int32_t* __restrict__ halo_begin,
                                                   int32_t* __restrict__ halo) {
    __shared__ int32_t keys[MAX_RING], cnts[MAX_RING], skey[MAX_RING], scnt[MAX_RING], off[MAX_RING + 1];
    __shared__ int32_t nring;
    int32_t t = blockIdx.x;
    if (t >= ntile) return;
    int o[3], s[3];
    tile_box(b, bits, tlist[t], o, s);
    const int ex = s[0] + 2, ey = s[1] + 2, ez = b.dim == 3 ? s[2] + 2 : 1;
    if (threadIdx.x == 0) nring = 0;
    __syncthreads();
    for (int bc = threadIdx.x; bc < ex * ey * ez; bc += BLK) {
        int r[3] = {bc % ex, (bc / ex) % ey, bc / (ex * ey)};
        bool interior = r[0] >= 1 && r[0] <= s[0] && r[1] >= 1 && r[1] <= s[1] &&
                        (b.dim == 2 || (r[2] >= 1 && r[2] <= s[2]));
        if (interior) continue;
        int cc[3] = {0, 0, 0};
        bool ok = true;
        for (int a = 0; a < b.dim; ++a) {
            int x = o[a] - 1 + r[a];
            if (b.periodic[a]) x = x < 0 ? x + b.nc[a] : (x >= b.nc[a] ? x - b.nc[a] : x);
            else if (x < 0 || x >= b.nc[a]) ok = false;
            cc[a] = x;
        }
        if (!ok) continue;
        int32_t key = cell_key(b, cc[0], cc[1], cc[2]);
        int32_t cnt = cell_start[key + 1] - cell_start[key];
        if (cnt == 0) continue;
        int idx = atomicAdd(&nring, 1);
        keys[idx] = key;
        cnts[idx] = cnt;
    }
    __syncthreads();
    const int R = nring;
    for (int a = threadIdx.x; a < R; a += BLK) {
        int rank = 0;
        int32_t ka = keys[a];
        for (int q = 0; q < R; ++q) rank += keys[q] < ka ? 1 : 0;
        skey[rank] = ka;
        scnt[rank] = cnts[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int q = 0; q < R; ++q) {
            off[q] = acc;
            acc += scnt[q];
        }
        off[R] = acc;
        if (PASS == 0) halo_cnt[t] = acc;
    }
    __syncthreads();
    if (PASS == 1) {
        int32_t base = halo_begin[t];
        for (int q = threadIdx.x; q < R; q += BLK) {
            int32_t s0 = cell_start[skey[q]];
            for (int e = 0; e < scnt[q]; ++e) halo[base + off[q] + e] = s0 + e;
        }
    }
}

// One thread per sorted slot: the tasks of its row.  PASS 0 counts them;
// PASS 1 writes them, with the record of the partner (own or halo) and the
// row entry of the mirrored pair.  err[0] counts partners that were not
// found (a broken invariant: the neighbour relation is symmetric and the
// ring holds every neighbour).
template <int DIM, int PASS>
__global__ void k_tile_tasks(int32_t n, int bits, BoxArgs b, const float4* __restrict__ sorted,
                             const int32_t* __restrict__ tidx, const int4* __restrict__ info,
                             const int32_t* __restrict__ halo, const int64_t* __restrict__ rp_s,
                             const int32_t* __restrict__ col_s, int32_t* __restrict__ cnt,
                             const int64_t* __restrict__ task_ptr, uint2* __restrict__ tasks, int32_t* err) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 pp = sorted[i];
    int cx = cell_coord(pp.x, b.lo[0], b.inv_cell[0], b.nc[0]);
    int cy = cell_coord(pp.y, b.lo[1], b.inv_cell[1], b.nc[1]);
    int cz = DIM == 3 ? cell_coord(pp.z, b.lo[2], b.inv_cell[2], b.nc[2]) : 0;
    int32_t T = cell_key(b, cx, cy, cz) >> bits;
    int4 ti = info[tidx[T]];
    const int32_t ob = ti.x, oc = ti.y, hb = ti.z, hc = ti.w;
    const int32_t p = i - ob;
    const int64_t kb = rp_s[ob];
    const int64_t k0 = rp_s[i], k1 = rp_s[i + 1];
    int64_t w = PASS ? task_ptr[i] : 0;
    int32_t c = 0;
    int32_t bad = 0;
    for (int64_t k = k0; k < k1; ++k) {
        int32_t j = col_s[k];
        bool own = (uint32_t)(j - ob) < (uint32_t)oc;
        if (own && j - ob < p) continue;
        if (PASS) {
            uint32_t q, mk = 0xffffu;
            if (own) {
                q = (uint32_t)(j - ob);
                int64_t m0 = rp_s[j], m1 = rp_s[j + 1], kk = -1;
                for (int64_t a = m0; a < m1; ++a)
                    if (col_s[a] == i) {
                        kk = a;
                        break;
                    }
                if (kk < 0) ++bad;
                mk = (uint32_t)(kk - kb);
            } else {
                int32_t lo = 0, hi = hc;  // first halo entry >= j
                while (lo < hi) {
                    int32_t mid = (lo + hi) >> 1;
                    if (halo[hb + mid] < j) lo = mid + 1;
                    else hi = mid;
                }
                if (lo >= hc || halo[hb + lo] != j) ++bad;
                q = (uint32_t)(oc + lo);
            }
            tasks[w + c] = make_uint2((uint32_t)p | (q << 16), (uint32_t)(k - kb) | (mk << 16));
        }
        ++c;
    }
    if (!PASS) cnt[i] = c;
    if (PASS && bad) atomicAdd(err, bad);
}

__global__ void k_tile_pack(int32_t ntile, const int32_t* __restrict__ own_begin, const int32_t* __restrict__ own_cnt,
                            const int32_t* __restrict__ halo_begin, const int32_t* __restrict__ halo_cnt,
                            int4* __restrict__ info) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    info[t] = make_int4(own_begin[t], own_cnt[t], halo_begin[t], halo_cnt[t]);
}

__global__ void k_tile_hdr(int32_t ntile, const int4* __restrict__ info, const int64_t* __restrict__ rp_s,
                           const int64_t* __restrict__ task_ptr, const float4* __restrict__ sorted,
                           TileHdr* __restrict__ hdr) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    int4 ti = info[t];
    TileHdr h;
    h.ob = ti.x;
    h.oc = ti.y;
    h.hb = ti.z;
    h.hc = ti.w;
    h.kb = rp_s[ti.x];
    h.rows = (int32_t)(rp_s[ti.x + ti.y] - h.kb);
    h.tb = task_ptr[ti.x];
    h.ntask = (int32_t)(task_ptr[ti.x + ti.y] - h.tb);
    h.pad0 = h.pad1 = 0;
    float4 o = sorted[ti.x];
    h.ox = o.x;
    h.oy = o.y;
    h.oz = o.z;
    h.ow = 0.f;
    hdr[t] = h;
}

// Largest LDS need of a tile, its record count and row-entry count.
__global__ void k_tile_need(int32_t ntile, const int4* __restrict__ info, const int64_t* __restrict__ rp_s,
                            int rec_bytes, int row_bytes, int32_t* out) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    int4 ti = info[t];
    int64_t rows = rp_s[ti.x + ti.y] - rp_s[ti.x];
    int64_t rec = (int64_t)ti.y + ti.w;
    int64_t bytes = rec * rec_bytes + rows * row_bytes;
    atomicMax(&out[0], (int32_t)(bytes < INT32_MAX ? bytes : INT32_MAX));
    atomicMax(&out[1], (int32_t)(rec < INT32_MAX ? rec : INT32_MAX));
    atomicMax(&out[2], (int32_t)(rows < INT32_MAX ? rows : INT32_MAX));
    atomicMax(&out[3], ti.y);
}

// Whether a tile of 2^bits keys fits the grid: on a periodic axis the tile
// and its ring, measured from any point of the tile, must stay within half
// the box (so relative positions are the minimum images), i.e. nc >= 2s+5.
bool tile_fits_grid(const BoxArgs& b, int bits) {
    for (int a = 0; a < b.dim; ++a) {
        int s = tile_side(bits, b.dim, a);
        if (b.periodic[a] && b.nc[a] < 2 * s + 5) return false;
    }
    return true;
}

// Estimated LDS bytes of a typical tile (uniform density, 30% margin).
double tile_estimate(const sph_ctx* c, int bits, int rec_bytes, int row_bytes) {
    const BoxArgs& b = c->box;
    double cells = 1.0, box = 1.0, grid = 1.0;
    for (int a = 0; a < b.dim; ++a) {
        int s = tile_side(bits, b.dim, a);
        if (s > b.nc[a]) s = b.nc[a];
        cells *= s;
        box *= s + 2;
        grid *= b.nc[a];
    }
    double ppc = c->n / grid;
    double per_row = c->n > 0 ? (double)c->nnz / c->n : 0.0;
    return 1.3 * (ppc * box * rec_bytes + ppc * cells * per_row * row_bytes);
}

// Build scratch, freed (after the device is idle) when it goes out of scope.
struct TmpBuf : DevBuf {
    ~TmpBuf() {
        if (p) (void)hipDeviceSynchronize();
        release();
    }
};

int build_tiles(sph_ctx* c, int bits, int rec_bytes, int row_bytes, int32_t* need) {
    TileSet& ts = c->tiles;
    ts.valid = false;
    const BoxArgs& b = c->box;
    const int32_t n = c->n;
    const int32_t nT = (int32_t)(c->ncell >> bits);
    TmpBuf flag, tidx, tlist, ob, oc, hb, hc, cnt;
    SPH_HIP(c, flag.ensure((size_t)nT * 4));
    SPH_HIP(c, tidx.ensure((size_t)(nT + 1) * 4));
    hipLaunchKernelGGL(k_tile_flags, dim3(grid_for(nT, BLK)), dim3(BLK), 0, c->stream, nT, bits,
                       c->cell_start.as<int32_t>(), flag.as<int32_t>());
    SPH_LAUNCH_CHECK(c);
    int r = sph_scan_i32_to_i32(c, flag.as<int32_t>(), tidx.as<int32_t>(), nT);
    if (r) return r;
    int32_t ntile = 0;
    SPH_HIP(c, hipMemcpyAsync(&ntile, tidx.as<int32_t>() + nT, 4, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    const size_t nt1 = (size_t)(ntile > 0 ? ntile : 1) + 1;
    SPH_HIP(c, tlist.ensure(nt1 * 4));
    SPH_HIP(c, ob.ensure(nt1 * 4));
    SPH_HIP(c, oc.ensure(nt1 * 4));
    SPH_HIP(c, hb.ensure(nt1 * 4));
    SPH_HIP(c, hc.ensure(nt1 * 4));
    hipLaunchKernelGGL(k_tile_list, dim3(grid_for(nT, BLK)), dim3(BLK), 0, c->stream, nT, bits, flag.as<int32_t>(),
                       tidx.as<int32_t>(), c->cell_start.as<int32_t>(), tlist.as<int32_t>(), ob.as<int32_t>(),
                       oc.as<int32_t>());
    hipLaunchKernelGGL(k_tile_ring<0>, dim3(ntile), dim3(BLK), 0, c->stream, ntile, bits, b,
                       c->cell_start.as<int32_t>(), tlist.as<int32_t>(), hc.as<int32_t>(), nullptr, nullptr);
    SPH_LAUNCH_CHECK(c);
    r = sph_scan_i32_to_i32(c, hc.as<int32_t>(), hb.as<int32_t>(), ntile);
    if (r) return r;
    int32_t nhalo = 0;
    SPH_HIP(c, hipMemcpyAsync(&nhalo, hb.as<int32_t>() + ntile, 4, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    SPH_HIP(c, ts.halo.ensure((size_t)(nhalo > 0 ? nhalo : 1) * 4));
    hipLaunchKernelGGL(k_tile_ring<1>, dim3(ntile), dim3(BLK), 0, c->stream, ntile, bits, b,
                       c->cell_start.as<int32_t>(), tlist.as<int32_t>(), nullptr, hb.as<int32_t>(),
                       ts.halo.as<int32_t>());
    SPH_HIP(c, ts.info.ensure(nt1 * sizeof(int4)));
    hipLaunchKernelGGL(k_tile_pack, dim3(grid_for(ntile, BLK)), dim3(BLK), 0, c->stream, ntile, ob.as<int32_t>(),
                       oc.as<int32_t>(), hb.as<int32_t>(), hc.as<int32_t>(), ts.info.as<int4>());
    SPH_LAUNCH_CHECK(c);

    // tasks
    SPH_HIP(c, cnt.ensure((size_t)n * 4));
    SPH_HIP(c, ts.task_ptr.ensure((size_t)(n + 1) * 8));
    auto tasks = [&](auto pass) {
        constexpr int P = decltype(pass)::value;
        if (c->dim == 2)
            hipLaunchKernelGGL((k_tile_tasks<2, P>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, bits, b,
                               c->sorted.as<float4>(), tidx.as<int32_t>(), ts.info.as<int4>(), ts.halo.as<int32_t>(),
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), cnt.as<int32_t>(),
                               ts.task_ptr.as<int64_t>(), ts.tasks.as<uint2>(), c->counter.as<int32_t>());
        else
            hipLaunchKernelGGL((k_tile_tasks<3, P>), dim3(grid_for(n, BLK)), dim3(BLK), 0, c->stream, n, bits, b,
                               c->sorted.as<float4>(), tidx.as<int32_t>(), ts.info.as<int4>(), ts.halo.as<int32_t>(),
                               c->rp_s.as<int64_t>(), c->col_s.as<int32_t>(), cnt.as<int32_t>(),
                               ts.task_ptr.as<int64_t>(), ts.tasks.as<uint2>(), c->counter.as<int32_t>());
    };
    tasks(std::integral_constant<int, 0>{});
    SPH_LAUNCH_CHECK(c);
    r = sph_scan_i32_to_i64(c, cnt.as<int32_t>(), ts.task_ptr.as<int64_t>(), n);
    if (r) return r;
    int64_t ntask = 0;
    SPH_HIP(c, hipMemcpyAsync(&ntask, ts.task_ptr.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    SPH_HIP(c, ts.tasks.ensure((size_t)(ntask > 0 ? ntask : 1) * sizeof(uint2)));
    SPH_HIP(c, c->counter.ensure(64));
    SPH_HIP(c, hipMemsetAsync(c->counter.p, 0, 64, c->stream));
    tasks(std::integral_constant<int, 1>{});
    hipLaunchKernelGGL(k_tile_need, dim3(grid_for(ntile, BLK)), dim3(BLK), 0, c->stream, ntile, ts.info.as<int4>(),
                       c->rp_s.as<int64_t>(), rec_bytes, row_bytes, c->counter.as<int32_t>() + 4);
    SPH_HIP(c, ts.hdr.ensure(nt1 * sizeof(TileHdr)));
    hipLaunchKernelGGL(k_tile_hdr, dim3(grid_for(ntile, BLK)), dim3(BLK), 0, c->stream, ntile, ts.info.as<int4>(),
                       c->rp_s.as<int64_t>(), ts.task_ptr.as<int64_t>(), c->sorted.as<float4>(),
                       ts.hdr.as<TileHdr>());
    SPH_LAUNCH_CHECK(c);
    int32_t h[8];
    SPH_HIP(c, hipMemcpyAsync(h, c->counter.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    if (h[0] != 0)
        return sph_fail(c, SPH_ERR_STATE, "cell tiles: %d neighbour pairs not found in a tile (broken invariant)", h[0]);
    for (int a = 0; a < 4; ++a) need[a] = h[4 + a];
    ts.bits = bits;
    ts.ntile = ntile;
    ts.ntask = ntask;
    ts.rec_bytes = rec_bytes;
    ts.row_bytes = row_bytes;
    ts.max_lds = need[0];
    ts.max_own = need[3];
    ts.max_rec = need[1];
    return SPH_OK;
}

}  // namespace

int sph_tiles_prepare(sph_ctx* c, int rec_bytes, int row_bytes, int lds_budget) {
    TileSet& ts = c->tiles;
    if (ts.valid && ts.rec_bytes == rec_bytes && ts.row_bytes == row_bytes && ts.max_lds <= lds_budget) return SPH_OK;
    if (ts.failed && ts.rec_bytes == rec_bytes && ts.row_bytes == row_bytes && ts.budget == lds_budget) return 1;
    ts.valid = false;
    ts.failed = true;  // until a tile size fits
    ts.rec_bytes = rec_bytes;
    ts.row_bytes = row_bytes;
    ts.budget = lds_budget;
    const BoxArgs& b = c->box;
    if (!b.morton || c->n == 0) return 1;
    const int lo = b.dim == 2 ? 2 : 3, hi = b.dim == 2 ? 8 : 9;
    int maxbits = 0;  // the key space bounds the tile size
    while (((int64_t)1 << (maxbits + 1)) <= c->ncell && maxbits + 1 <= hi) ++maxbits;
    // tuning override: SPH_TILE_BITS
    int forced = 0;
    if (const char* e = getenv("SPH_TILE_BITS")) forced = atoi(e);
    int first = forced >= lo && forced <= maxbits ? forced : maxbits;
    for (int bits = first; bits >= lo; --bits) {
        if (!tile_fits_grid(b, bits)) continue;
        if (!forced && tile_estimate(c, bits, rec_bytes, row_bytes) > lds_budget) continue;
        int32_t need[4];
        int r = build_tiles(c, bits, rec_bytes, row_bytes, need);
        if (r) return r;
        if (need[0] <= lds_budget && need[1] < 65535 && need[2] < 65535) {
            ts.valid = true;
            ts.failed = false;
            if (getenv("SPH_TILE_VERBOSE"))
                fprintf(stderr,
                        "[sph tiles] n=%d bits=%d tiles=%d tasks=%lld nnz=%lld max_lds=%d max_rec=%d max_rows=%d "
                        "max_own=%d\n",
                        c->n, bits, ts.ntile, (long long)ts.ntask, (long long)c->nnz, need[0], need[1], need[2],
                        need[3]);
            return SPH_OK;
        }
        if (forced) break;
    }
    return 1;
}
