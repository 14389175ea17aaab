// Uniform-grid binning of the point clouds by a device counting sort:
// bounding box, grid parameters, then a partition of the points into
// buckets of consecutive cells and a per-bucket sort by cell in LDS.
// The grid is the spatial index the flooding and landmark kernels scan; it
// replaces the paper's presorted axis slices and Boolean masks (Sec. 4.2 and
// its appendix) with cell lists that are contiguous in memory.
#include "internal.hpp"

namespace flood {

static constexpr int kBlock = 256;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
static int grid_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}
hipError_t fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(n)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_blocks(n)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}
__global__ void k_copy_u32b(const uint32_t *src, uint32_t *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}
hipError_t copy_u32(const uint32_t *src, uint32_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_u32b, dim3(grid_blocks(n)), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_blocks(n)), dim3(kBlock), 0, s, p, v, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (3 phases; 1024 threads x 4 items per block)
static constexpr int kScanThreads = 1024;
static constexpr int kScanItems = 4;
static constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_tmp_elems(int64_t n) {
    // every recursion level stores its block sums followed by 4 spare slots
    size_t tot = 0;
    int64_t m = n;
    do {
        m = (m + kScanTile - 1) / kScanTile;
        tot += (size_t)m + 4;
    } while (m > 1);
    return tot + 64;
}

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t warp_sums[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) warp_sums[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint32_t w = lane < kScanThreads / 64 ? warp_sums[lane] : 0u;
        uint32_t z = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(z, o, 64);
            if (lane >= o) z += y;
        }
        if (lane < kScanThreads / 64) warp_sums[lane] = z - w;
        if (lane == kScanThreads / 64 - 1) *total = z;
    }
    __syncthreads();
    uint32_t r = warp_sums[wid] + x - v;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_local(uint32_t *d, int64_t n, uint32_t *block_sums) {
    __shared__ uint32_t tot;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? d[base + i] : 0u;
        s += v[i];
    }
    uint32_t off = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) d[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint32_t *d, int64_t n, const uint32_t *block_off) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t a = block_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) d[base + i] += a;
}

hipError_t exclusive_scan_u32(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    uint32_t *sums = tmp;
    uint32_t *sums2 = tmp + nb + 4;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    if (nb > 1) {
        hipError_t e = exclusive_scan_u32(sums, nb, sums2, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grid build

// blocks per cloud of the bounding-box pass (each writes one partial box)
static int bbox_blocks(int32_t B, const int64_t *x_off) {
    int64_t nmax = 0;
    for (int32_t b = 0; b < B; ++b) nmax = nmax > x_off[b + 1] - x_off[b] ? nmax : x_off[b + 1] - x_off[b];
    int64_t bx = (nmax + kBlock * 8 - 1) / (kBlock * 8);
    return (int)(bx < 1 ? 1 : (bx > 1024 ? 1024 : bx));
}

// partition shape: blocks per cloud and cells per bucket (a cloud's bucket
// counters and a bucket's cell counters both live in LDS)
static constexpr int kPartTile = 8192;      // points per partition block, about
static constexpr int kSortBlock = 1024;     // threads of a bucket-sort block
static constexpr int kPU = 4;               // points a thread handles at once
static constexpr int kMaxBuckets = 16384;   // buckets per cloud
static constexpr int kMinShift = 10, kMaxShift = 15;
struct PartShape {
    int32_t bx, shift;
    int64_t nbtot, nbmax;
    bool ok;
};
static PartShape part_shape(int32_t B, const int64_t *x_off, float alpha) {
    PartShape ps;
    int64_t nmax = 0, capmax = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = x_off[b + 1] - x_off[b];
        nmax = n > nmax ? n : nmax;
        const int64_t cap = cells_cap(n, alpha);
        capmax = cap > capmax ? cap : capmax;
    }
    int shift = kMinShift;
    while (shift < kMaxShift && ((capmax + (1ll << shift) - 1) >> shift) > kMaxBuckets) ++shift;
    ps.shift = shift;
    ps.ok = ((capmax + (1ll << shift) - 1) >> shift) <= kMaxBuckets;
    int64_t bx = (nmax + kPartTile - 1) / kPartTile;
    ps.bx = (int32_t)(bx < 1 ? 1 : (bx > 1024 ? 1024 : bx));
    ps.nbtot = 0;
    ps.nbmax = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t nb = (cells_cap(x_off[b + 1] - x_off[b], alpha) + (1ll << shift) - 1) >> shift;
        ps.nbtot += nb;
        ps.nbmax = nb > ps.nbmax ? nb : ps.nbmax;
    }
    return ps;
}

size_t grid_workspace(int32_t B, const int64_t *x_off, float alpha, int64_t *total_cells) {
    int64_t tc = 0;
    for (int32_t b = 0; b < B; ++b) tc += cells_cap(x_off[b + 1] - x_off[b], alpha);
    if (total_cells) *total_cells = tc;
    const PartShape ps = part_shape(B, x_off, alpha);
    int64_t np = x_off[B];
    size_t bytes = 0;
    bytes += sizeof(GridParam) * B + 256;
    bytes += sizeof(uint32_t) * 6 * B + 256;
    bytes += sizeof(float) * 6 * (size_t)B * bbox_blocks(B, x_off) + 256;
    bytes += sizeof(float4) * np + 256;                        // xs
    bytes += sizeof(uint32_t) * (tc + 1) + 256;                // cell_start
    bytes += sizeof(uint32_t) * (tc / 32 + 2) + 256;           // occupancy bits
    bytes += sizeof(float4) * np + 256;                        // tmp_pt
    bytes += sizeof(uint32_t) * (ps.nbtot + 1) + 256;          // bucket counts, then starts
    bytes += sizeof(uint32_t) * ps.nbtot + 256;                // bucket cursors
    bytes += sizeof(uint32_t) * scan_tmp_elems(ps.nbtot + 1) + 256;
    bytes += sizeof(int64_t) * (B + 1) + 256;                  // bk_off
    return bytes;
}

void grid_carve(Carve &c, int32_t B, const int64_t *x_off, float alpha, GridWork &g) {
    const int64_t total_pts = x_off[B];
    int64_t tc = 0;
    for (int32_t b = 0; b < B; ++b) tc += cells_cap(x_off[b + 1] - x_off[b], alpha);
    const PartShape ps = part_shape(B, x_off, alpha);
    g.gp = c.take<GridParam>(B);
    g.bbox = c.take<uint32_t>(6 * (size_t)B);
    g.bbox_blocks = bbox_blocks(B, x_off);
    g.bbox_part = c.take<float>(6 * (size_t)B * g.bbox_blocks);
    g.xs = c.take<float4>(total_pts);
    g.cell_start = c.take<uint32_t>(tc + 1);
    g.occ = c.take<uint32_t>(tc / 32 + 2);
    g.tmp_pt = c.take<float4>(total_pts);
    g.bstart = c.take<uint32_t>(ps.nbtot + 1);
    g.bcursor = c.take<uint32_t>(ps.nbtot);
    g.scan_tmp = c.take<uint32_t>(scan_tmp_elems(ps.nbtot + 1));
    g.bk_off = c.take<int64_t>(B + 1);
    g.bx = ps.ok ? ps.bx : 0;  // 0: a cloud needs more cells than the partition supports
    g.shift = ps.shift;
    g.nbtot = ps.nbtot;
    g.nbmax = ps.nbmax;
    g.total_cells = tc;
    g.total_pts = total_pts;
}

// gridDim.y = cloud; block x reduces a strided share of the cloud and
// writes its partial box (no atomics: thousands of blocks would contend on
// six words)
__global__ __launch_bounds__(kBlock) void k_bbox(const float *X, const int64_t *x_off, float *part) {
    const int b = blockIdx.y;
    const int64_t lo = x_off[b], hi = x_off[b + 1];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = X[3 * i + a];
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
    }
    __shared__ float s_mn[3][kBlock / 64], s_mx[3][kBlock / 64];
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            s_mn[a][wid] = mn[a];
            s_mx[a][wid] = mx[a];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        float *o = part + 6 * ((int64_t)b * gridDim.x + blockIdx.x);
        for (int a = 0; a < 3; ++a) {
            float m0 = s_mn[a][0], m1 = s_mx[a][0];
            for (int w = 1; w < kBlock / 64; ++w) {
                m0 = fminf(m0, s_mn[a][w]);
                m1 = fmaxf(m1, s_mx[a][w]);
            }
            o[a] = m0;
            o[3 + a] = m1;
        }
    }
}

// one block per cloud: the box of the partial boxes, as ordered keys
__global__ __launch_bounds__(kBlock) void k_bbox_final(const float *part, int nblk, uint32_t *bbox) {
    const int b = blockIdx.x;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
        const float *p = part + 6 * ((int64_t)b * nblk + i);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], p[a]);
            mx[a] = fmaxf(mx[a], p[3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], o, 64));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], o, 64));
        }
    }
    __shared__ float s_mn[3][kBlock / 64], s_mx[3][kBlock / 64];
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            s_mn[a][wid] = mn[a];
            s_mx[a][wid] = mx[a];
        }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            float m0 = s_mn[a][0], m1 = s_mx[a][0];
            for (int w = 1; w < kBlock / 64; ++w) {
                m0 = fminf(m0, s_mn[a][w]);
                m1 = fmaxf(m1, s_mx[a][w]);
            }
            bbox[6 * b + a] = float_key(m0);
            bbox[6 * b + 3 + a] = float_key(m1);
        }
}

// grid parameters of every cloud, one thread per cloud in rounds of a
// block; the cell bases and bucket offsets are prefix sums over the clouds
__global__ __launch_bounds__(1024) void k_grid_params(const uint32_t *bbox, const int64_t *x_off, int32_t B,
                                                       float alpha, int32_t max_dim, int64_t morton_lo,
                                                       int64_t morton_hi, int32_t shift, GridParam *gp,
                                                       int64_t *bk_off) {
    int64_t cell_carry = 0, bk_carry = 0;
    for (int32_t b0 = 0; b0 < B; b0 += (int32_t)blockDim.x) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        GridParam g;
        int64_t cap = 0, nbk = 0;
        if (b < B) {
            int64_t n = x_off[b + 1] - x_off[b];
            cap = cells_cap(n, alpha);
            nbk = (cap + (1ll << shift) - 1) >> shift;
            float lo[3], hi[3], e[3];
            float emax = 0.f, amax = 0.f;
            for (int a = 0; a < 3; ++a) {
                lo[a] = key_float(bbox[6 * b + a]);
                hi[a] = key_float(bbox[6 * b + 3 + a]);
                if (!(lo[a] <= hi[a])) { lo[a] = 0.f; hi[a] = 0.f; }  // empty cloud or non-finite data
                e[a] = hi[a] - lo[a];
                emax = fmaxf(emax, e[a]);
                amax = fmaxf(amax, fmaxf(fabsf(lo[a]), fabsf(hi[a])));
            }
            if (!(emax > 0.f)) emax = 1.f;
            double target = (double)(cap - 64) > 1.0 ? (double)(cap - 64) : 1.0;
            double vol = 1.0;
            for (int a = 0; a < 3; ++a) vol *= fmax((double)e[a], 1e-7 * (double)emax);
            double h = cbrt(vol / target);
            if (!(h > 0.0)) h = emax;
            int64_t nx = 1, ny = 1, nz = 1;
            g.morton = (n >= morton_lo && n < morton_hi) ? 1 : 0;
            if (g.morton) {
                // a 2^m cube over the largest extent, 8^m <= cap - 64 cells
                int m = 0;
                while (m < 10 && ((int64_t)8 << (3 * m)) <= cap - 64 && ((int64_t)2 << m) <= max_dim) ++m;
                nx = ny = nz = (int64_t)1 << m;
                h = (double)emax / (double)nx;
            } else {
                for (int it = 0; it < 4096; ++it) {
                    nx = (int64_t)floor((double)e[0] / h) + 1;
                    ny = (int64_t)floor((double)e[1] / h) + 1;
                    nz = (int64_t)floor((double)e[2] / h) + 1;
                    if (nx <= max_dim && ny <= max_dim && nz <= max_dim && nx * ny * nz <= cap) break;
                    h *= 1.05;
                }
            }
            g.ox = lo[0]; g.oy = lo[1]; g.oz = lo[2];
            g.h = (float)h;
            g.inv_h = (float)(1.0 / h);
            g.eps = 1e-3f * (float)h + 1e-6f * amax;
            g.nx = (int32_t)nx; g.ny = (int32_t)ny; g.nz = (int32_t)nz;
            g.pt_base = x_off[b];
            g.npts = n;
            g.cells_cap = cap;
        }
        int64_t cells_total, bk_total;
        const int64_t cell_off = block_exclusive_i64(cap, cells_total);
        const int64_t bk_of = block_exclusive_i64(nbk, bk_total);
        if (b < B) {
            g.cell_base = cell_carry + cell_off;
            gp[b] = g;
            bk_off[b] = bk_carry + bk_of;
        }
        cell_carry += cells_total;
        bk_carry += bk_total;
    }
    if (threadIdx.x == 0) bk_off[B] = bk_carry;
}


// global cell of a point (the binning rule of the grid)
__device__ __forceinline__ uint32_t point_cell(float x, float y, float z, const GridParam &g) {
    const int cx = bin_coord(x, g.ox, g.inv_h, g.nx);
    const int cy = bin_coord(y, g.oy, g.inv_h, g.ny);
    const int cz = bin_coord(z, g.oz, g.inv_h, g.nz);
    return g.morton ? (uint32_t)g.cell_base + (spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2))
                    : (uint32_t)(g.cell_base + ((int64_t)cz * g.ny + cy) * g.nx + cx);
}

// points [lo, hi) of cloud b handled by partition block x
__device__ __forceinline__ void part_range(const GridParam &g, int x, int bx, int64_t &lo, int64_t &hi) {
    const int64_t tile = (g.npts + bx - 1) / bx;
    lo = g.pt_base + (int64_t)x * tile;
    hi = g.pt_base + g.npts;
    if (lo + tile < hi) hi = lo + tile;
}

// counts of this block's points per bucket of its cloud, in LDS
__device__ __forceinline__ void part_local_count(const float *X, const GridParam &g, int64_t lo, int64_t hi,
                                                 int32_t shift, uint32_t *s_h) {
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kBlock * kPU) {
        uint32_t j[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            j[u] = i < hi ? (point_cell(X[3 * i], X[3 * i + 1], X[3 * i + 2], g) - (uint32_t)g.cell_base) >> shift : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (i0 + (int64_t)u * kBlock < hi) atomicAdd(&s_h[j[u]], 1u);
    }
}

// gridDim = (bx, B): bucket sizes (block counts added per nonzero bucket)
__global__ __launch_bounds__(kBlock) void k_part_count(const float *X, const GridParam *gp, const int64_t *bk_off,
                                                        int32_t shift, uint32_t *bcount) {
    extern __shared__ uint32_t s_h[];
    const int b = blockIdx.y, x = blockIdx.x, bx = gridDim.x;
    const GridParam g = gp[b];
    const int64_t g0 = bk_off[b], nb = bk_off[b + 1] - g0;
    for (int64_t j = threadIdx.x; j < nb; j += kBlock) s_h[j] = 0u;
    __syncthreads();
    int64_t lo, hi;
    part_range(g, x, bx, lo, hi);
    part_local_count(X, g, lo, hi, shift, s_h);
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nb; j += kBlock)
        if (s_h[j]) atomicAdd(&bcount[g0 + j], s_h[j]);
}

// gridDim = (bx, B): the block claims a run in each bucket it feeds (one
// atomic per bucket) and moves its points there (positions from LDS)
__global__ __launch_bounds__(kBlock) void k_part_scatter(const float *X, const GridParam *gp, const int64_t *bk_off,
                                                          int32_t shift, uint32_t *bcursor, float4 *tmp_pt) {
    extern __shared__ uint32_t s_h[];
    const int b = blockIdx.y, x = blockIdx.x, bx = gridDim.x;
    const GridParam g = gp[b];
    const int64_t g0 = bk_off[b], nb = bk_off[b + 1] - g0;
    for (int64_t j = threadIdx.x; j < nb; j += kBlock) s_h[j] = 0u;
    __syncthreads();
    int64_t lo, hi;
    part_range(g, x, bx, lo, hi);
    part_local_count(X, g, lo, hi, shift, s_h);
    __syncthreads();
    for (int64_t j = threadIdx.x; j < nb; j += kBlock)
        if (s_h[j]) s_h[j] = atomicAdd(&bcursor[g0 + j], s_h[j]);
    __syncthreads();
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kBlock * kPU) {
        float4 v[kPU];
        uint32_t pos[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i < hi) v[u] = make_float4(X[3 * i], X[3 * i + 1], X[3 * i + 2], __int_as_float((int)i));
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (i0 + (int64_t)u * kBlock < hi)
                pos[u] = atomicAdd(&s_h[(point_cell(v[u].x, v[u].y, v[u].z, g) - (uint32_t)g.cell_base) >> shift], 1u);
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (i0 + (int64_t)u * kBlock < hi) tmp_pt[pos[u]] = v[u];
    }
}

// exclusive scan of n <= NT * per values in LDS, in place (per: values per thread)
template <int NT>
__device__ void lds_exclusive_scan(uint32_t *v, int n, int per) {
    __shared__ uint32_t s_w[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int a = tid * per, e = min(a + per, n);
    uint32_t sum = 0;
    for (int k = a; k < e; ++k) sum += v[k];
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[wid] = incl;
    __syncthreads();
    uint32_t off = incl - sum;
    for (int w = 0; w < wid; ++w) off += s_w[w];
    for (int k = a; k < e; ++k) {
        const uint32_t t = v[k];
        v[k] = off;
        off += t;
    }
    __syncthreads();
}

// one block per bucket: its points sorted by cell, its cells' starts
__global__ __launch_bounds__(kSortBlock) void k_bucket_sort(const GridParam *gp, const int64_t *bk_off, int32_t B,
                                                             int32_t shift, const uint32_t *bstart,
                                                             const float4 *tmp_pt, uint32_t *cell_start, float4 *xs,
                                                             int64_t nbtot, int64_t total_cells, int64_t total_pts) {
    extern __shared__ uint32_t s_c[];
    const int64_t gb = blockIdx.x;
    int lo = 0, hi = B;  // cloud: the last b with bk_off[b] <= gb
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bk_off[mid] <= gb) lo = mid;
        else hi = mid;
    }
    const GridParam g = gp[lo];
    const int64_t c0 = g.cell_base + ((gb - bk_off[lo]) << shift);
    const int64_t cend = g.cell_base + g.cells_cap;
    const int ncell = (int)((c0 + (1ll << shift) < cend ? c0 + (1ll << shift) : cend) - c0);
    const uint32_t p0 = bstart[gb], p1 = bstart[gb + 1];
    for (int k = threadIdx.x; k < ncell; k += kSortBlock) s_c[k] = 0u;
    __syncthreads();
    for (uint32_t q = p0 + threadIdx.x; q < p1; q += kSortBlock * kPU) {
        uint32_t c[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const uint32_t p = q + u * kSortBlock;
            if (p < p1) {
                const float4 v = tmp_pt[p];
                c[u] = point_cell(v.x, v.y, v.z, g) - (uint32_t)c0;
            }
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (q + u * kSortBlock < p1) atomicAdd(&s_c[c[u]], 1u);
    }
    __syncthreads();
    lds_exclusive_scan<kSortBlock>(s_c, ncell, (ncell + kSortBlock - 1) / kSortBlock);
    for (int k = threadIdx.x; k < ncell; k += kSortBlock) cell_start[c0 + k] = p0 + s_c[k];
    if (gb == nbtot - 1 && threadIdx.x == 0) cell_start[total_cells] = (uint32_t)total_pts;
    __syncthreads();
    for (uint32_t q = p0 + threadIdx.x; q < p1; q += kSortBlock * kPU) {
        float4 v[kPU];
        uint32_t c[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const uint32_t p = q + u * kSortBlock;
            if (p < p1) {
                v[u] = tmp_pt[p];
                c[u] = point_cell(v[u].x, v[u].y, v[u].z, g) - (uint32_t)c0;
            }
        }
#pragma unroll
        for (int u = 0; u < kPU; ++u)
            if (q + u * kSortBlock < p1) xs[p0 + atomicAdd(&s_c[c[u]], 1u)] = v[u];
    }
}

// one lane per cell: a wave's ballot gives the occupancy bits of its 64
// consecutive cells, i.e. two words
__global__ __launch_bounds__(kBlock) void k_occ_bits(const uint32_t *cell_start, int64_t total_cells, uint32_t *occ) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool held = c < total_cells && cell_start[c + 1] > cell_start[c];
    const uint64_t m = __ballot(held);
    if ((threadIdx.x & 63) == 0 && c < total_cells) {
        occ[c >> 5] = (uint32_t)m;
        if (c + 32 < total_cells) occ[(c >> 5) + 1] = (uint32_t)(m >> 32);
    }
}

hipError_t grid_build(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                      float alpha, GridWork &g, hipStream_t s, int32_t max_dim, int64_t morton_lo, int64_t morton_hi) {
    (void)x_off;
    if (g.bx < 1) return hipErrorInvalidValue;  // a cloud with more cells than the partition supports
    hipLaunchKernelGGL(k_bbox, dim3(g.bbox_blocks, B), dim3(kBlock), 0, s, X, x_off_d, g.bbox_part);
    hipLaunchKernelGGL(k_bbox_final, dim3(B), dim3(kBlock), 0, s, g.bbox_part, g.bbox_blocks, g.bbox);
    hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(1024), 0, s, g.bbox, x_off_d, B, alpha, max_dim, morton_lo, morton_hi,
                       g.shift, g.gp, g.bk_off);
    hipError_t e = fill_u32(g.bstart, 0u, g.nbtot + 1, s);
    if (e != hipSuccess) return e;
    const size_t sh_part = sizeof(uint32_t) * (size_t)g.nbmax;
    hipLaunchKernelGGL(k_part_count, dim3(g.bx, B), dim3(kBlock), sh_part, s, X, g.gp, g.bk_off, g.shift, g.bstart);
    e = exclusive_scan_u32(g.bstart, g.nbtot + 1, g.scan_tmp, s);
    if (e != hipSuccess) return e;
    e = copy_u32(g.bstart, g.bcursor, g.nbtot, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_part_scatter, dim3(g.bx, B), dim3(kBlock), sh_part, s, X, g.gp, g.bk_off, g.shift, g.bcursor,
                       g.tmp_pt);
    const size_t sh_bucket = sizeof(uint32_t) << g.shift;
    if (sh_bucket > 65536) {
        e = hipFuncSetAttribute((const void *)k_bucket_sort, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh_bucket);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_bucket_sort, dim3((unsigned)g.nbtot), dim3(kSortBlock), sh_bucket, s, g.gp, g.bk_off, B,
                       g.shift, g.bstart, g.tmp_pt, g.cell_start, g.xs, g.nbtot, g.total_cells, g.total_pts);
    hipLaunchKernelGGL(k_occ_bits, dim3((unsigned)((g.total_cells + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       g.cell_start, g.total_cells, g.occ);
    return hipGetLastError();
}

}  // namespace flood
