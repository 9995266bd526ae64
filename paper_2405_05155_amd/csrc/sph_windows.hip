// sph_windows.hip -- neighbour windows of the pair loops over fixed-stride
// rows (the 3-D Eulerian stage and the total-Lagrangian stress divergence).
//
// The slots of one workgroup, block b = [b P, b P + P) of the cell-sorted
// order, reference a few hundred distinct neighbours (on the 200^3 lattice
// at 1.6h about 4.6 per own particle for P = 128).  The window of block b
// lists its own slots first, in order, then the distinct other slots its
// rows reference, ascending; the rows are rewritten as 16-bit positions in
// that list.  A workgroup copies its window's records into LDS once and its
// pairs then read them there instead of gathering each neighbour through
// the vector cache.  Built once per configuration.
#include "sph_internal.h"

#include <cstdlib>
#include <cstring>

namespace {

constexpr int BLK = 256;
constexpr int WIN_HASH = 4096;  // open-addressing set of a block's distinct neighbours (LDS)

// Exclusive scan of one value per thread over the workgroup (BLK threads);
// returns the exclusive prefix and stores the total in *total.
__device__ int32_t wg_exclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < BLK; o <<= 1) {
        const int32_t u = (int32_t)threadIdx.x >= o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += u;
        __syncthreads();
    }
    const int32_t incl = lds[threadIdx.x];
    *total = lds[BLK - 1];
    __syncthreads();
    return incl - v;
}

// Pass 1 (list == nullptr): window length of every block into len[b] and the
// longest into *maxlen (a block with more than WIN_HC_MAX distinct
// neighbours reports WIN_HC_MAX + 1).  Pass 2: the windows into
// list[off[b] ..] and the rows into colw as 16 times the window position
// (the record's byte offset in an LDS plane).  Rows are padded from S to Sp
// entries with the slot itself (a zero-weight pair), so that each of the L
// lanes of a slot takes a whole number of chunks of M entries; entry
// k = s + L (c M + t) of slot i (lane s, chunk c, t < M) sits at
// colw[((c n + i) L + s) M + t], so a lane loads a chunk at once.  The distinct other slots are collected in an
// LDS hash set (linear probing, at most WIN_HASH probes per insertion),
// then compacted and sorted (bitonic).
__global__ void __launch_bounds__(BLK) k_window(int32_t n, int32_t S, int32_t Sp, int32_t P, int32_t L, int32_t M,
                                                const int32_t* __restrict__ colE, int32_t* __restrict__ len,
                                                int32_t* __restrict__ maxlen, const int32_t* __restrict__ off,
                                                int32_t* __restrict__ list, uint16_t* __restrict__ colw) {
    __shared__ int32_t T[WIN_HASH];
    __shared__ int32_t a[WIN_HASH];
    __shared__ int32_t lds_scan[BLK];
    __shared__ int32_t distinct;
    const int32_t b = (int32_t)blockIdx.x;
    const int32_t b0 = b * P;
    const int32_t own = min(P, n - b0);
    for (int32_t t = threadIdx.x; t < WIN_HASH; t += BLK) T[t] = -1;
    if (threadIdx.x == 0) distinct = 0;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < P * S; t += BLK) {
        const int32_t e = t / P, pp = t - e * P;
        if (pp >= own) continue;
        const int32_t v = colE[(int64_t)e * n + b0 + pp];
        if (v >= b0 && v < b0 + own) continue;
        if (*(volatile int32_t*)&distinct > WIN_HC_MAX) continue;  // too long already: stop inserting
        uint32_t h = ((uint32_t)v * 2654435761u) >> 20;  // 12 bits
        for (int probe = 0; probe < WIN_HASH; ++probe) {
            const int32_t old = atomicCAS(&T[h], -1, v);
            if (old == -1) {
                atomicAdd(&distinct, 1);
                break;
            }
            if (old == v) break;
            h = (h + 1) & (WIN_HASH - 1);
        }
    }
    __syncthreads();
    const int32_t others = distinct;
    if (others + own > WIN_HC_MAX) {
        if (!list && threadIdx.x == 0) {
            len[b] = WIN_HC_MAX + 1;
            atomicMax(maxlen, WIN_HC_MAX + 1);
        }
        return;
    }
    if (!list) {
        if (threadIdx.x == 0) {
            len[b] = own + others;
            atomicMax(maxlen, own + others);
        }
        return;
    }
    // compact the set into a[0 .. others), then sort it
    constexpr int C = WIN_HASH / BLK;
    int32_t m = 0;
#pragma unroll
    for (int q = 0; q < C; ++q) m += T[threadIdx.x * C + q] != -1 ? 1 : 0;
    int32_t total;
    int32_t at = wg_exclusive_scan(m, lds_scan, &total);
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const int32_t v = T[threadIdx.x * C + q];
        if (v != -1) a[at++] = v;
    }
    int32_t E2 = 2;
    while (E2 < others) E2 <<= 1;
    __syncthreads();
    for (int32_t t = others + (int32_t)threadIdx.x; t < E2; t += BLK) a[t] = INT32_MAX;
    __syncthreads();
    for (int32_t k = 2; k <= E2; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t t = threadIdx.x; t < E2 / 2; t += BLK) {
                const int32_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const int32_t hi = lo + j;
                const int32_t x = a[lo], y = a[hi];
                if ((x > y) == ((lo & k) == 0)) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    int32_t* out = list + off[b];
    for (int32_t t = threadIdx.x; t < own + others; t += BLK) out[t] = t < own ? b0 + t : a[t - own];
    for (int32_t t = threadIdx.x; t < P * Sp; t += BLK) {
        const int32_t e = t / P, pp = t - e * P;
        if (pp >= own) continue;
        const int32_t v = e < S ? colE[(int64_t)e * n + b0 + pp] : b0 + pp;
        const int32_t ls = e % L, lj = e / L;
        const int64_t at2 = (((int64_t)(lj / M) * n + b0 + pp) * L + ls) * M + lj % M;
        int32_t pos;
        if (v >= b0 && v < b0 + own) {
            pos = v - b0;
        } else {
            int32_t lo = 0, hi = others;  // first index with a[index] >= v
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (a[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            pos = own + lo;
        }
        colw[at2] = (uint16_t)(pos << 4);
    }
}

// Pairs per chunk of a lane: the M in {6, 8, 10, 12} whose chunks cover mu
// entries with the fewest padding pairs (the larger on a tie).
int window_chunk(int mu) {
    const int cand[4] = {12, 10, 8, 6};
    int best = 12, cost = 1 << 30;
    for (int M : cand) {
        const int k = (mu + M - 1) / M * M;
        if (k < cost) cost = k, best = M;
    }
    return best;
}

}  // namespace

int sph_windows_prepare(sph_ctx* c, NeighbourWindows& w, int L, int P) {
    if (w.state != 0 && w.P == P && w.L == L) return SPH_OK;
    w.state = -1;
    w.P = P;
    w.L = L;
    const int32_t n = c->n, S = c->ell_S;
    if (c->ell_state != 1 || n <= 0 || S <= 0 || L < 1 || P < 1) return SPH_OK;
    const int mu = (S + L - 1) / L;
    const int M = window_chunk(mu);
    const int32_t Sp = (mu + M - 1) / M * M * L;
    if ((double)Sp * n >= 1073741824.0) return SPH_OK;  // 32-bit entry offsets
    const int32_t nb = (n + P - 1) / P;
    SPH_HIP(c, w.len.ensure((size_t)nb * sizeof(int32_t)));
    SPH_HIP(c, w.off.ensure(((size_t)nb + 1) * sizeof(int32_t)));
    SPH_HIP(c, c->counter.ensure(64));
    SPH_HIP(c, hipMemsetAsync(c->counter.p, 0, 4, c->stream));
    hipLaunchKernelGGL(k_window, dim3((unsigned)nb), dim3(BLK), 0, c->stream, n, S, Sp, P, L, M,
                       c->colE.as<int32_t>(), w.len.as<int32_t>(), c->counter.as<int32_t>(), nullptr, nullptr,
                       nullptr);
    SPH_LAUNCH_CHECK(c);
    int r = sph_scan_i32_to_i32(c, w.len.as<int32_t>(), w.off.as<int32_t>(), nb);
    if (r) return r;
    int32_t host[2] = {0, 0};
    SPH_HIP(c, hipMemcpyAsync(&host[0], c->counter.p, 4, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipMemcpyAsync(&host[1], w.off.as<int32_t>() + nb, 4, hipMemcpyDeviceToHost, c->stream));
    SPH_HIP(c, hipStreamSynchronize(c->stream));
    if (host[0] > WIN_HC_MAX) return SPH_OK;
    SPH_HIP(c, w.list.ensure((size_t)host[1] * sizeof(int32_t)));
    SPH_HIP(c, w.col.ensure((size_t)Sp * n * sizeof(uint16_t)));
    hipLaunchKernelGGL(k_window, dim3((unsigned)nb), dim3(BLK), 0, c->stream, n, S, Sp, P, L, M,
                       c->colE.as<int32_t>(), nullptr, nullptr, w.off.as<int32_t>(), w.list.as<int32_t>(),
                       w.col.as<uint16_t>());
    SPH_LAUNCH_CHECK(c);
    w.max = host[0];
    w.M = M;
    w.Sp = Sp;
    w.state = 1;
    return SPH_OK;
}
