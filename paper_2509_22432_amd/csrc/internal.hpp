// Internal declarations shared by the HIP translation units of libflood.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/flood.h"

namespace flood {

// Per-cloud uniform grid.  Cell (ix,iy,iz) of cloud b is global cell
// cell_base + (iz*ny + iy)*nx + ix, or cell_base + morton(ix,iy,iz) on a
// 2^m cube when `morton` is set (landmark grids of large clouds, whose
// sorted order must be spatially compact); cell_start[] holds global
// positions in the cell-sorted point array, so one exclusive scan serves
// every cloud.
struct GridParam {
    float ox, oy, oz;   // grid origin (bbox minimum)
    float h, inv_h;     // cell edge and its reciprocal
    float eps;          // slack added around cell boxes (covers rounding of the binning)
    int32_t nx, ny, nz; // cells per axis
    int32_t morton;     // 1: cells numbered in Morton order (nx = ny = nz = 2^m)
    int64_t cell_base;  // first global cell of this cloud
    int64_t pt_base;    // first global point of this cloud
    int64_t npts;
    int64_t cells_cap;  // cells reserved for this cloud
};

// workspace carving helper: 256-byte aligned sub-buffers
struct Carve {
    uintptr_t base, cur, end;
    explicit Carve(void *p, size_t n) : base((uintptr_t)p), cur((uintptr_t)p), end((uintptr_t)p + n) {}
    template <class T> T *take(size_t count) {
        cur = (cur + 255) & ~(uintptr_t)255;
        T *r = (T *)cur;
        cur += count * sizeof(T);
        return r;
    }
    size_t used() const { return (size_t)(cur - base) + 256; }
    bool ok() const { return cur <= end; }
};

// cells reserved per cloud: ceil(alpha * n) + 64 (same formula host and device)
__host__ __device__ inline int64_t cells_cap(int64_t n, float alpha) {
    double c = (double)alpha * (double)n;
    return (int64_t)c + 1 + 64;
}

// Exclusive prefix sum over a block: thread t passes v (its item's value)
// and receives the sum of the values of threads 0..t-1; every thread gets
// the block total.  Called by every thread of a block of at most 1024.
__device__ inline int64_t block_exclusive_i64(int64_t v, int64_t &total) {
    // Hillis-Steele inclusive scan in LDS, log2(blockDim) rounds
    __shared__ int64_t s_part[1024];
    const unsigned t = threadIdx.x;
    s_part[t] = v;
    __syncthreads();
    for (unsigned off = 1; off < blockDim.x; off <<= 1) {
        const int64_t x = t >= off ? s_part[t - off] : 0;
        __syncthreads();
        s_part[t] += x;
        __syncthreads();
    }
    const int64_t incl = s_part[t];
    total = s_part[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Ordered-key encoding of floats for atomic min/max on unsigned ints.
__device__ inline uint32_t float_key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// 10-bit value with its bits spread to every third position (Morton codes)
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000ff;
    v = (v | (v << 8)) & 0x0300f00f;
    v = (v | (v << 4)) & 0x030c30c3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// cell coordinate of a coordinate value (the binning rule; NaN maps to 0,
// +inf and values past the grid to n - 1)
__device__ inline int bin_coord(float v, float o, float inv_h, int n) {
    const float t = (v - o) * inv_h;
    return (t >= 0.f) ? (t < (float)n ? (int)t : n - 1) : 0;
}

// any occupied cell among global cells [a, b] (a <= b), from the occupancy bits
__device__ __forceinline__ bool any_occupied(const uint32_t *__restrict__ occ, int64_t a, int64_t b) {
    const int64_t w0 = a >> 5, w1 = b >> 5;
    for (int64_t w = w0; w <= w1; ++w) {
        uint32_t m = occ[w];
        if (w == w0) m &= 0xffffffffu << (a & 31);
        if (w == w1) m &= 0xffffffffu >> (31 - (b & 31));
        if (m) return true;
    }
    return false;
}

// ---- wave primitives (DPP) ----
// DPP lane moves within rows of 16 lanes (quad_perm xor 1, xor 2, then the
// half-row and row mirrors): after the four steps every lane of a row holds
// the row's reduction; the four rows are combined through scalar reads
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t rd_lane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_max_u32(uint32_t v) { return max(v, dpp_mov<CTRL>(v)); }
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min_u32(uint32_t v) { return min(v, dpp_mov<CTRL>(v)); }

// the lane holding the wave's largest key (mb << 32) | ~id: the largest mb,
// and among equal mb the lowest id (all 64 lanes active); mmax gets that mb
__device__ __forceinline__ int wave_argmax_key(uint32_t mb, uint32_t id, uint32_t &mmax) {
    uint32_t v = dpp_max_u32<0x140>(dpp_max_u32<0x141>(dpp_max_u32<0x4e>(dpp_max_u32<0xb1>(mb))));
    mmax = max(max(rd_lane(v, 0), rd_lane(v, 16)), max(rd_lane(v, 32), rd_lane(v, 48)));
    const uint64_t tied = __ballot(mb == mmax);
    if (__popcll(tied) == 1) return __ffsll((unsigned long long)tied) - 1;
    uint32_t u = mb == mmax ? id : 0xffffffffu;
    u = dpp_min_u32<0x140>(dpp_min_u32<0x141>(dpp_min_u32<0x4e>(dpp_min_u32<0xb1>(u))));
    const uint32_t umin = min(min(rd_lane(u, 0), rd_lane(u, 16)), min(rd_lane(u, 32), rd_lane(u, 48)));
    return __ffsll((unsigned long long)__ballot(mb == mmax && id == umin)) - 1;
}

__device__ __forceinline__ float wave_max_f32_dpp(float v) {
    v = fmaxf(v, __uint_as_float(dpp_mov<0xb1>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dpp_mov<0x4e>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dpp_mov<0x141>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dpp_mov<0x140>(__float_as_uint(v))));
    const float a = fmaxf(__uint_as_float(rd_lane(__float_as_uint(v), 0)), __uint_as_float(rd_lane(__float_as_uint(v), 16)));
    const float b = fmaxf(__uint_as_float(rd_lane(__float_as_uint(v), 32)), __uint_as_float(rd_lane(__float_as_uint(v), 48)));
    return fmaxf(a, b);
}

__device__ __forceinline__ float wave_min_f32_dpp(float v) {
    v = fminf(v, __uint_as_float(dpp_mov<0xb1>(__float_as_uint(v))));
    v = fminf(v, __uint_as_float(dpp_mov<0x4e>(__float_as_uint(v))));
    v = fminf(v, __uint_as_float(dpp_mov<0x141>(__float_as_uint(v))));
    v = fminf(v, __uint_as_float(dpp_mov<0x140>(__float_as_uint(v))));
    const float a = fminf(__uint_as_float(rd_lane(__float_as_uint(v), 0)), __uint_as_float(rd_lane(__float_as_uint(v), 16)));
    const float b = fminf(__uint_as_float(rd_lane(__float_as_uint(v), 32)), __uint_as_float(rd_lane(__float_as_uint(v), 48)));
    return fminf(a, b);
}

// inclusive prefix sum over the wave (rows of 16 by DPP shifts, then the
// row broadcasts of lanes 15 and 31); all 64 lanes active
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_add_u32(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    v = dpp_add_u32<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add_u32<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add_u32<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add_u32<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add_u32<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add_u32<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// the lane holding the wave's smallest (mb, id) pair (all 64 lanes active);
// mmin gets that mb
__device__ __forceinline__ int wave_argmin_pair(uint32_t mb, uint32_t id, uint32_t &mmin) {
    uint32_t v = dpp_min_u32<0x140>(dpp_min_u32<0x141>(dpp_min_u32<0x4e>(dpp_min_u32<0xb1>(mb))));
    mmin = min(min(rd_lane(v, 0), rd_lane(v, 16)), min(rd_lane(v, 32), rd_lane(v, 48)));
    const uint64_t tied = __ballot(mb == mmin);
    if (__popcll(tied) == 1) return __ffsll((unsigned long long)tied) - 1;
    uint32_t u = mb == mmin ? id : 0xffffffffu;
    u = dpp_min_u32<0x140>(dpp_min_u32<0x141>(dpp_min_u32<0x4e>(dpp_min_u32<0xb1>(u))));
    const uint32_t umin = min(min(rd_lane(u, 0), rd_lane(u, 16)), min(rd_lane(u, 32), rd_lane(u, 48)));
    return __ffsll((unsigned long long)__ballot(mb == mmin && id == umin)) - 1;
}

// ---- grid build (grid.hip) ----
// The counting sort by cell runs in two partition passes with no atomics on
// cells: cells are grouped per cloud in buckets of 2^shift consecutive
// cells; bx blocks per cloud count and move their share of the points per
// bucket (one device atomic per block and bucket it feeds), then one block
// per bucket sorts its points by cell in LDS.
struct GridWork {
    GridParam *gp;        // [B]
    uint32_t *bbox;       // [B][6] ordered keys: min xyz, max xyz
    float *bbox_part;     // [B][bbox_blocks][6] partial boxes
    int bbox_blocks;
    float4 *xs;           // [sum N] (x, y, z, bits of global point row), sorted by cell
    uint32_t *cell_start; // [total_cells + 1]
    uint32_t *occ;        // [total_cells / 32 + 1] bit c set: cell c holds points
    float4 *tmp_pt;       // [sum N] points grouped by bucket
    uint32_t *bstart;     // [nbtot + 1] bucket sizes, then bucket starts
    uint32_t *bcursor;    // [nbtot] bucket fill cursors
    uint32_t *scan_tmp;   // block sums for the scan of bstart
    int64_t *bk_off;      // [B + 1] first bucket of each cloud
    int32_t bx;           // partition blocks per cloud
    int32_t shift;        // log2 of the cells per bucket
    int64_t nbtot;        // buckets over all clouds
    int64_t nbmax;        // buckets of the largest cloud
    int64_t total_cells;
    int64_t total_pts;
};
size_t grid_workspace(int32_t B, const int64_t *x_off, float alpha, int64_t *total_cells);
void grid_carve(Carve &c, int32_t B, const int64_t *x_off, float alpha, GridWork &g);
hipError_t grid_build(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                      float alpha, GridWork &g, hipStream_t s, int32_t max_dim = 1 << 20,
                      int64_t morton_lo = INT64_MAX, int64_t morton_hi = INT64_MAX);

// generic helpers (grid.hip)
hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
hipError_t fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t copy_u32(const uint32_t *src, uint32_t *dst, int64_t n, hipStream_t s);
hipError_t exclusive_scan_u32(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);

// ---- farthest-point sampling (fps.hip) ----
size_t fps_workspace(int32_t B, const int64_t *x_off, const int32_t *n_lm);
hipError_t fps_run(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                   const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                   float *radius, void *ws, size_t ws_bytes, hipStream_t s);

// ---- flooding (flood.hip) ----
struct FloodSizes {
    int64_t n[4];        // simplices per dimension (n[0] = landmarks)
    int64_t total_pts;
    int64_t total_cells;
};
size_t flood_workspace(const flood_problem *pb, float alpha, FloodSizes *sz);
hipError_t flood_run(const flood_problem *pb, const flood_tuning &tu, const flood_outputs *out,
                     void *ws, size_t ws_bytes, hipStream_t s);

// ---- backward (backward.hip) ----
hipError_t backward_run(const flood_problem *pb, const flood_outputs *fwd, const float *const grad_f[4],
                        float *grad_X, float *grad_L, hipStream_t s);

}  // namespace flood
