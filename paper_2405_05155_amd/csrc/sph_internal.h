// sph_internal.h -- context, scratch buffers and device helpers shared by the
// HIP translation units of libsph.  Not installed; the public ABI is sph.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/sph.h"

// ------------------------------------------------------------------ host side

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need) {
        if (need <= bytes && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t b = need < 256 ? 256 : need;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Per-axis geometry passed by value to kernels.
struct BoxArgs {
    float lo[3];
    float L[3];
    float halfL[3];
    float inv_cell[3];  // nc / L
    int nc[3];
    int periodic[3];
    double Ld[3];       // FP64 box lengths for the exact neighbour test
    double halfLd[3];
    int dim;
    int morton;         // 1: cell keys are Morton codes; 0: linear (z, y, x)
};

// Cell keys.  Morton (Z-order) codes of the cell coordinates keep cells that
// are close in space close in the cell-sorted particle array; the linear
// key is the fallback for grids whose Morton key space would be too large.
__host__ __device__ __forceinline__ uint32_t spread2(uint32_t x) {  // 16 bits -> even bits
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t x) {  // 10 bits -> every third bit
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
__host__ __device__ __forceinline__ int32_t cell_key(const BoxArgs& b, int x, int y, int z) {
    if (b.morton) {
        if (b.dim == 2) return (int32_t)(spread2((uint32_t)x) | (spread2((uint32_t)y) << 1));
        return (int32_t)(spread3((uint32_t)x) | (spread3((uint32_t)y) << 1) | (spread3((uint32_t)z) << 2));
    }
    return (z * b.nc[1] + y) * b.nc[0] + x;
}

// Load element idx of an array through a 32-bit byte offset from a uniform
// base (one shift per gather; needs idx * sizeof(T) < 2^32).
template <class T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}

// Cell coordinate of a position on one axis (clamped to the grid).
__host__ __device__ __forceinline__ int cell_coord(float x, float lo, float inv, int nc) {
    int c = (int)floorf((x - lo) * inv);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Workgroups are handed to the 8 XCDs of the chip round-robin; remapping
// the block index gives XCD k one contiguous range of the cell-sorted
// particles, so each XCD's L2 holds the neighbourhood of its own region.
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nb) {
    const int32_t X = 8;
    int32_t per = nb / X, rem = nb % X;
    int32_t x = b % X, k = b / X;
    return x * per + (x < rem ? x : rem) + k;
}

// Longest window the pair kernels' LDS planes hold.
constexpr int WIN_HC_MAX = 1024;

// Neighbour windows of blocks of P consecutive cell-sorted slots over the
// fixed-stride rows: per block its own slots, in order, then the distinct
// other slots its rows reference, ascending (`list`, offsets `off`), and the
// rows as 16-bit LDS byte offsets (16 x window position), padded with the
// slot itself to whole chunks of M entries for each of the L lanes of a slot:
// entry s + L (c M + t) of slot i (lane s, chunk c, t < M) at
// col[((c n + i) L + s) M + t].
struct NeighbourWindows {
    int state = 0;        // 0: not built, 1: valid, -1: not used for this configuration
    int P = 0;            // slots per block
    int L = 0;            // lanes per slot
    int M = 0;            // entries per chunk
    int32_t Sp = 0;       // row entries after padding
    int32_t max = 0;      // longest window
    DevBuf len;           // int32 [nblocks]
    DevBuf off;           // int32 [nblocks + 1]
    DevBuf list;          // int32 [off[nblocks]]
    DevBuf col;           // uint16 [Sp n]
};

struct sph_ctx {
    int dim = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    char err[1024] = {0};

    // bound configuration
    bool bound = false;
    sph_domain dom{};
    int32_t n = 0;
    double rc = 0.0, rc2 = 0.0;
    BoxArgs box{};
    int64_t ncell = 0;
    int64_t nnz = 0;

    DevBuf pos4;        // float4 [n] (x, y, z, 0), caller order
    DevBuf cell_of;     // int32 [n]
    DevBuf slot;        // int32 [n]
    DevBuf cell_start;  // int32 [ncell + 1]
    DevBuf sorted;      // float4 [n] (x, y, z, bits(index)) in cell order
    DevBuf sorted_tmp;  // float4 [n] provisional placement before the in-cell ordering
    DevBuf cnt;         // int32 [n]
    DevBuf row_ptr;     // int64 [n + 1]   caller order (export)
    DevBuf col;         // int32 [nnz]     caller order, caller indices, rows ascending (built on export)
    bool export_valid = false;
    DevBuf cnt_s;       // int32 [n]       per cell-sorted slot
    DevBuf rp_s;        // int64 [n + 1]   cell-sorted rows
    DevBuf col_s;       // int32 [nnz]     cell-sorted rows, sorted-slot indices
    DevBuf scan_tmp;    // block sums of the scans
    DevBuf counter;     // small device counters / reductions

    // cached corrected geometry: (position, V, B upper triangle)
    bool geo_valid = false;
    DevBuf geo0;  // float4 [n]: 3-D (x, y, z, V); 2-D (x, y, V, B00)
    DevBuf geo1;  // float4 [n]: 3-D (B00, B01, B02, B11); 2-D float2 (B01, B11)
    DevBuf geo2;  // float2 [n]: 3-D (B12, B22)
    uint64_t geo_gen = 0;        // bumped whenever geo0..geo2 change or go stale
    DevBuf rec3;                 // 3-D Eulerian stage records: two sets of float4 [4n] (geometry and state)

    // state scratch
    DevBuf ua, ub;      // float4 [n] packed states
    DevBuf ta, tb, tc;  // misc per-particle scratch
    DevBuf fa, fb, fc;  // total Lagrangian: F in cell-sorted order (float4, float4, float)
    DevBuf pa;          // total Lagrangian: current positions in cell-sorted order (float4)

    // relaxation: exterior-tail table and reductions
    DevBuf tail;        // float [ntail]
    double tail_h = 0.0, tail_R = 0.0;
    int ntail = 0, tail_kernel = -1;
    DevBuf svol;        // cell-order scratch: volumes (pair loops) or (x, y, z, V) records (relaxation)
    DevBuf sfield;      // float [n] a caller field in cell order
    DevBuf partials;    // per-block reduction partials
    DevBuf relax_scalars;

    int num_cu = 0;     // compute units of the device (filled on first use)

    int euler_path = SPH_PATH_NONE;  // variant the last Eulerian call ran
    int tlsph_path = SPH_PATH_NONE;  // variant of kernel B in the last total-Lagrangian call

    // fixed-stride neighbour rows over cell-sorted slots (ELLPACK): entry k
    // of slot i at colE[k * n + i] for k < ell_S, rows shorter than ell_S
    // padded with i itself (a zero-weight pair); built on first use when the
    // padding stays small
    DevBuf colE;
    int32_t ell_S = 0;
    int ell_state = 0;  // 0: not built, 1: valid, -1: rows too uneven (CSR is used)

    // neighbour windows over the fixed-stride rows (sph_windows_prepare):
    // the 3-D Eulerian stage's and the total-Lagrangian kernels'
    NeighbourWindows win3, wtl;
};

// Build (or reuse) the fixed-stride neighbour rows of the bound
// configuration.  Sets c->ell_state; returns an error code only on failure.
int sph_ell_prepare(sph_ctx* c);


int sph_fail(sph_ctx* c, int code, const char* fmt, ...);

// Build (or reuse) the windows w of blocks of P slots with L lanes per slot
// over the bound configuration's fixed-stride rows (two passes of one
// workgroup per block: an LDS hash set of the distinct neighbours, then
// their sorted list and the rewritten rows).  Sets w.state to 1, or to -1
// when the rows are not fixed-stride or a window would exceed WIN_HC_MAX
// records; returns an error code only on failure.
int sph_windows_prepare(sph_ctx* c, NeighbourWindows& w, int L, int P);

// Take the device address of sph_mlp_train_step_noalloc's fixed workspace on
// `device` (the current device), once per device.
void sph_mlp_noalloc_setup(int device);

#define SPH_HIP(ctx, expr)                                                                     \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return sph_fail((ctx), SPH_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

#define SPH_LAUNCH_CHECK(ctx)                                                                      \
    do {                                                                                           \
        hipError_t _e = hipGetLastError();                                                         \
        if (_e != hipSuccess)                                                                      \
            return sph_fail((ctx), SPH_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(_e)); \
    } while (0)

// validate the domain and bin positions into cells (no neighbour list)
int sph_bin_cells(sph_ctx* c, const sph_domain* dom, int32_t n, const float* pos);
// sph_bin_cells on cells at least kappa h / div wide, linear keys when `linear`
int sph_bin_cells_grid(sph_ctx* c, const sph_domain* dom, int32_t n, const float* pos, int div, bool linear);

// exclusive scan of int32 counts into int32 or int64 offsets, out[n] = total
int sph_scan_i32_to_i32(sph_ctx* c, const int32_t* in, int32_t* out, int64_t n);
int sph_scan_i32_to_i64(sph_ctx* c, const int32_t* in, int64_t* out, int64_t n);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ------------------------------------------------------------------ device side

// Compensated (Kahan) accumulator.  The running estimate of the sum is
// s - c (c holds the rounding error of the last addition, with sign).
struct Kahan {
    float s, c;
    __device__ __forceinline__ void init(float v = 0.f) { s = v; c = 0.f; }
    __device__ __forceinline__ void add(float x) {
        float y = x - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    // Terms taken two at a time (w1 x1 + w2 x2, one compensated addition
    // per two terms): open folds the first into the carried correction (c
    // then holds y = w1 x1 - c, rounded once, until the matching close),
    // close adds the second to y and y to the sum.
    __device__ __forceinline__ void open(float w, float x) { c = fmaf(w, x, -c); }
    __device__ __forceinline__ void close(float w, float x) {
        float y = fmaf(w, x, c);
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ float value() const { return s - c; }
};

// w x into a lane's compensated partial sum of one row.
__device__ __forceinline__ void accum(Kahan& k, float w, float x) { k.add(w * x); }

// v of lane (lane ^ m) of the wave: for m = 1 and 2 (partners within an
// aligned group of four lanes) a DPP quad permutation, which moves the value
// inside the vector ALU; otherwise through the LDS crossbar (ds_bpermute).
__device__ __forceinline__ float lane_xor(float v, int m) {
    if (m == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    if (m == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    return __shfl_xor(v, m, 64);
}

// v of the first lane of the lane's aligned group of four (DPP broadcast).
__device__ __forceinline__ float quad_first(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x00, 0xF, 0xF, false));
}

// Combine the compensated partial sums held by the L lanes of an aligned
// lane group (xor butterfly; every lane ends with the same value).  Each
// partial is the pair (hi, lo) = (s, -c); partners merge with TwoSum so the
// rounding error of adding the high parts is carried in the low part.
template <int L>
__device__ __forceinline__ float group_sum(const Kahan& k) {
    float hi = k.s, lo = -k.c;
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
        float ohi = lane_xor(hi, m);
        float olo = lane_xor(lo, m);
        float s = hi + ohi;
        float bp = s - hi;
        float e = (hi - (s - bp)) + (ohi - bp);
        lo = (lo + olo) + e;
        hi = s;
    }
    return hi + lo;
}

// group_sum keeping the combined (hi, lo) pair in FP64 (for sums that feed
// an FP64 computation).
template <int L>
__device__ __forceinline__ double group_sum64(const Kahan& k) {
    float hi = k.s, lo = -k.c;
#pragma unroll
    for (int m = 1; m < L; m <<= 1) {
        float ohi = lane_xor(hi, m);
        float olo = lane_xor(lo, m);
        float s = hi + ohi;
        float bp = s - hi;
        float e = (hi - (s - bp)) + (ohi - bp);
        lo = (lo + olo) + e;
        hi = s;
    }
    return (double)hi + (double)lo;
}

__device__ __forceinline__ float min_image(float d, float L, float halfL, int periodic) {
    if (periodic) {
        if (d > halfL) d -= L;
        else if (d < -halfL) d += L;
    }
    return d;
}

// Kernel constants (host computes them in FP64 once per call).
struct KernelConsts {
    float hinv;      // 1/h
    float cW;        // W normalisation: Wendland alpha_d; LG a_d / h^d
    float cF;        // (dW/dr)/r prefactor: Wendland -5 alpha_d / h^2; LG -a_d/(3 h^{d+2})
    int type;        // SPH_WENDLAND / SPH_LAGUERRE_GAUSS
};

// Wendland: W = cW (1 - q/2)^4 (2q + 1);  (dW/dr)/r = cF (1 - q/2)^3.
// LG:       W = cW (1 - q^2 + q^4/6) e^{-q^2};
//           (dW/dr)/r = cF e^{-q^2} (12 - 8 q^2 + q^4).
__device__ __forceinline__ float kernel_W(const KernelConsts& k, float q) {
    if (k.type == SPH_WENDLAND) {
        float t = 1.f - 0.5f * q;
        float t2 = t * t;
        return k.cW * t2 * t2 * (2.f * q + 1.f);
    }
    float q2 = q * q;
    return k.cW * (1.f - q2 + q2 * q2 * (1.f / 6.f)) * __expf(-q2);
}

__device__ __forceinline__ float kernel_F(const KernelConsts& k, float q) {
    if (k.type == SPH_WENDLAND) {
        float t = 1.f - 0.5f * q;
        return k.cF * t * t * t;
    }
    float q2 = q * q;
    return k.cF * __expf(-q2) * (12.f - 8.f * q2 + q2 * q2);
}

__device__ __forceinline__ float wendland_F(float q, float cF) {
    float t = 1.f - 0.5f * q;
    return cF * t * t * t;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

KernelConsts make_kernel_consts(int type, int dim, double h);
// Cell grid of the box: cells at least rc / div wide; Morton keys unless
// `linear` (or the Morton key space would be too large), else (z, y, x).
BoxArgs make_box_args(const sph_domain& d, double rc, int div = 1, bool linear = false);
int64_t cell_slots(const BoxArgs& b);  // size of the cell-key space

// ------------------------------------------------------------------ pair-loop helpers

// A lane's M entries of one chunk (M / 2 words of two 16-bit entries each,
// starting at word `at`), in as few loads as their alignment allows.
template <int M>
__device__ __forceinline__ void load_chunk(const uint16_t* __restrict__ colw, uint32_t at, uint32_t (&w)[M / 2]) {
    const uint32_t* p = reinterpret_cast<const uint32_t*>(colw);
    if constexpr (M == 8) {
        const uint4 v = ld32(reinterpret_cast<const uint4*>(p), at >> 2);
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (M == 12) {
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            const uint2 v = ld32(reinterpret_cast<const uint2*>(p), (at >> 1) + (uint32_t)h);
            w[2 * h] = v.x;
            w[2 * h + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int h = 0; h < M / 2; ++h) w[h] = ld32(p, at + (uint32_t)h);
    }
}

// Periodic geometry for the pair loops: wrap d - L rint(d / L) on periodic
// axes (invL = 0 elsewhere), needed only by waves holding a particle within
// `margin` of a periodic face.
struct Wrap {
    float L[3], invL[3], lo[3];
    float margin;
};

__device__ __forceinline__ float wrap1(float d, float L, float invL) { return fmaf(-L, rintf(d * invL), d); }

__device__ __forceinline__ bool wave_needs_wrap(const Wrap& w, const float4& x) {
    bool near = false;
    const float xs[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (w.invL[a] != 0.f) {
            const float off = xs[a] - w.lo[a];
            near = near || off < w.margin || w.L[a] - off < w.margin;
        }
    }
    return __any(near);
}

// Row entries of sorted slot i taken by lane `sub` of an L-lane group:
// entries sub, sub + L, ...  ELL (entry k at col[k n + i], k < S) or CSR.
template <bool ELL, int L>
__device__ __forceinline__ void row_range(int32_t i, int sub, int32_t n, const int64_t* __restrict__ rp, int32_t S,
                                          int64_t& k, int64_t& e, int64_t& stride) {
    if (ELL) {
        k = (int64_t)sub * n + i;
        stride = (int64_t)L * n;
        e = (int64_t)S * n;
    } else {
        k = rp[i] + sub;
        stride = L;
        e = rp[i + 1];
    }
}

inline Wrap make_wrap(const sph_ctx* c) {
    Wrap w{};
    for (int a = 0; a < 3; ++a) {
        w.L[a] = c->box.L[a];
        w.invL[a] = c->box.periodic[a] ? (float)(1.0 / c->box.Ld[a]) : 0.f;
        w.lo[a] = c->box.lo[a];
    }
    w.margin = (float)(c->rc * 1.001);
    return w;
}
