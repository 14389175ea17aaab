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
