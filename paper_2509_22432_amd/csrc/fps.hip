// Farthest-point landmark selection on the GPU (greedy k-centre; the paper
// selects landmarks this way, Sec. 2 and Table 1).  One kernel launch per
// round for all clouds at once.  A round only visits the grid cells within
// the current covering radius R of the newest landmark (no point farther
// than R can lower its running minimum, since every minimum is <= R^2), and
// keeps a three-level max hierarchy (brick of W cells -> row -> z-slab) so
// the argmax is recomputed only where minima changed.  The last block of a
// cloud to finish (atomic counter) reduces the slabs and picks the next
// landmark.  Ties go to the lowest point index via the packed key
// (minimum bits << 32) | (~index).
#include "internal.hpp"

namespace flood {

static constexpr int kFpsBlock = 256;
static constexpr int kBrick = 8;  // cells per brick along x

struct FpsState {
    int32_t cur;   // local index of the newest landmark
    float r2;      // current max of the running minima (covering radius squared)
    uint32_t done; // blocks finished in this round
    int32_t pad;
};

struct FpsWork {
    GridWork grid;
    float *mind;       // [sum N] running minima, in cell-sorted order
    uint64_t *brick;   // [total_cells] brick maxima, indexed by the brick's first cell
    uint64_t *row;     // [total_cells] row maxima, indexed by the row's first cell
    uint64_t *slab;    // [total_cells] slab maxima, indexed by the slab's first cell
    FpsState *state;   // [B]
    int64_t *l_off;    // [B+1]
};

static float fps_alpha() { return 1.0f; }

size_t fps_workspace(int32_t B, const int64_t *x_off, const int32_t *n_lm) {
    (void)n_lm;
    int64_t tc = 0;
    size_t bytes = grid_workspace(B, x_off, fps_alpha(), &tc);
    int64_t np = x_off[B];
    bytes += sizeof(float) * np + 256;
    bytes += 3 * (sizeof(uint64_t) * tc + 256);
    bytes += sizeof(FpsState) * B + 256;
    bytes += sizeof(int64_t) * (B + 1) + 256;
    return bytes + 1024;
}

// recipe of the landmark rule: every operation rounded to float32, no FMA
__device__ __forceinline__ float fps_d2(float px, float py, float pz, float lx, float ly, float lz) {
    float dx = __fsub_rn(px, lx);
    float dy = __fsub_rn(py, ly);
    float dz = __fsub_rn(pz, lz);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t load_glc(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fps_init(int32_t B, const int32_t *n_lm, const int64_t *start, FpsState *st,
                           int64_t *l_off, int32_t *idx) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t o = 0;
    for (int32_t b = 0; b < B; ++b) {
        l_off[b] = o;
        st[b].cur = start ? (int32_t)start[b] : 0;
        st[b].r2 = INFINITY;
        st[b].done = 0;
        idx[o] = st[b].cur;
        o += n_lm[b];
    }
    l_off[B] = o;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// box of cells that can hold a point within R of l (one cell of margin)
__device__ inline void fps_box(const GridParam &g, float lx, float ly, float lz, float r2, int lo[3], int hi[3]) {
    const int n[3] = {g.nx, g.ny, g.nz};
    const float o[3] = {g.ox, g.oy, g.oz};
    const float l[3] = {lx, ly, lz};
    if (!(r2 < INFINITY)) {
        for (int a = 0; a < 3; ++a) { lo[a] = 0; hi[a] = n[a] - 1; }
        return;
    }
    float R = sqrtf(r2);
    for (int a = 0; a < 3; ++a) {
        float tl = (l[a] - R - o[a]) * g.inv_h;
        float th = (l[a] + R - o[a]) * g.inv_h;
        tl = fminf(fmaxf(tl, -4.f), (float)n[a] + 4.f);
        th = fminf(fmaxf(th, -4.f), (float)n[a] + 4.f);
        lo[a] = clampi((int)floorf(tl) - 1, 0, n[a] - 1);
        hi[a] = clampi((int)floorf(th) + 1, 0, n[a] - 1);
    }
}

__global__ __launch_bounds__(kFpsBlock) void k_fps_round(
    int32_t t, const float *__restrict__ X, const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs,
    const float4 *__restrict__ xs, float *__restrict__ mind, uint64_t *__restrict__ brick, uint64_t *__restrict__ rowmax,
    uint64_t *__restrict__ slabmax, FpsState *__restrict__ st, const int32_t *__restrict__ n_lm,
    const int64_t *__restrict__ l_off, int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    const int b = blockIdx.y;
    if (t >= n_lm[b]) return;
    const GridParam g = gp[b];
    const int32_t cur = st[b].cur;
    const float r2 = st[b].r2;
    const int64_t lrow = g.pt_base + cur;
    const float lx = X[3 * lrow], ly = X[3 * lrow + 1], lz = X[3 * lrow + 2];
    int lo[3], hi[3];
    fps_box(g, lx, ly, lz, r2, lo, hi);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * wpb;
    const int64_t bny = hi[1] - lo[1] + 1;
    const int64_t nrows = bny * (hi[2] - lo[2] + 1);
    const int nbr = (g.nx + kBrick - 1) / kBrick;
    const int bx0 = lo[0] / kBrick, bx1 = hi[0] / kBrick;
    const uint32_t base_idx = (uint32_t)g.pt_base;
    for (int64_t r = wave; r < nrows; r += nwaves) {
        const int z = lo[2] + (int)(r / bny);
        const int y = lo[1] + (int)(r % bny);
        const int64_t rowcell = g.cell_base + ((int64_t)z * g.ny + y) * g.nx;
        uint64_t rmax = 0;
        for (int br = bx0; br <= bx1; ++br) {
            const int c0 = br * kBrick;
            const int c1 = min(g.nx, c0 + kBrick);
            const uint32_t p0 = cs[rowcell + c0], p1 = cs[rowcell + c1];
            uint64_t kmax = 0;
            for (uint32_t p = p0 + lane; p < p1; p += 64) {
                const float4 q = xs[p];
                const float d2 = fps_d2(q.x, q.y, q.z, lx, ly, lz);
                float m = mind[p];
                if (d2 < m) {
                    m = d2;
                    mind[p] = m;
                }
                const uint32_t li = (uint32_t)__float_as_int(q.w) - base_idx;
                const uint64_t key = ((uint64_t)__float_as_uint(m) << 32) | (uint64_t)(0xffffffffu - li);
                kmax = key > kmax ? key : kmax;
            }
            kmax = wave_max_u64(kmax);
            if (lane == 0) brick[rowcell + c0] = kmax;
            rmax = kmax > rmax ? kmax : rmax;
        }
        uint64_t other = 0;
        for (int br = lane; br < nbr; br += 64)
            if (br < bx0 || br > bx1) {
                uint64_t v = brick[rowcell + (int64_t)br * kBrick];
                other = v > other ? v : other;
            }
        other = wave_max_u64(other);
        rmax = other > rmax ? other : rmax;
        if (lane == 0) rowmax[rowcell] = rmax;
    }
    // last block of this cloud reduces the touched slabs, then all slabs
    __shared__ uint32_t s_last;
    __shared__ uint64_t s_red[kFpsBlock / 64];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&st[b].done, 1u) == gridDim.x - 1) ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const int wid = threadIdx.x >> 6;
    for (int z = lo[2]; z <= hi[2]; ++z) {
        uint64_t m = 0;
        const int64_t slabcell = g.cell_base + (int64_t)z * g.ny * g.nx;
        for (int y = threadIdx.x; y < g.ny; y += blockDim.x) {
            uint64_t v = load_glc(&rowmax[slabcell + (int64_t)y * g.nx]);
            m = v > m ? v : m;
        }
        m = wave_max_u64(m);
        if (lane == 0) s_red[wid] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t v = 0;
            for (int w = 0; w < wpb; ++w) v = s_red[w] > v ? s_red[w] : v;
            __hip_atomic_store(&slabmax[slabcell], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
    uint64_t m = 0;
    for (int z = threadIdx.x; z < g.nz; z += blockDim.x) {
        uint64_t v = load_glc(&slabmax[g.cell_base + (int64_t)z * g.ny * g.nx]);
        m = v > m ? v : m;
    }
    m = wave_max_u64(m);
    if (lane == 0) s_red[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t v = 0;
        for (int w = 0; w < wpb; ++w) v = s_red[w] > v ? s_red[w] : v;
        const float best = __uint_as_float((uint32_t)(v >> 32));
        const int32_t nxt = (int32_t)(0xffffffffu - (uint32_t)(v & 0xffffffffu));
        const int64_t o = l_off[b];
        if (radius) radius[o + t] = __fsqrt_rn(best);
        if (t + 1 < n_lm[b]) idx_out[o + t + 1] = nxt;
        st[b].cur = nxt;
        st[b].r2 = best;
        st[b].done = 0;
    }
}

hipError_t fps_run(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                   const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                   float *radius, void *ws, size_t ws_bytes, hipStream_t s) {
    int64_t tc = 0;
    grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    Carve c(ws, ws_bytes);
    FpsWork w;
    grid_carve(c, B, np, tc, w.grid);
    w.mind = c.take<float>(np);
    w.brick = c.take<uint64_t>(tc);
    w.row = c.take<uint64_t>(tc);
    w.slab = c.take<uint64_t>(tc);
    w.state = c.take<FpsState>(B);
    w.l_off = c.take<int64_t>(B + 1);
    if (!c.ok()) return hipErrorOutOfMemory;
    hipError_t e = grid_build(X, B, x_off, x_off_d, fps_alpha(), w.grid, s);
    if (e != hipSuccess) return e;
    e = fill_f32(w.mind, INFINITY, np, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fps_init, dim3(1), dim3(1), 0, s, B, n_lm_d, start_d, w.state, w.l_off, idx);
    int64_t nmax = 0;
    int32_t rounds = 0;
    for (int32_t b = 0; b < B; ++b) {
        nmax = x_off[b + 1] - x_off[b] > nmax ? x_off[b + 1] - x_off[b] : nmax;
        rounds = n_lm[b] > rounds ? n_lm[b] : rounds;
    }
    int bpc = (int)((nmax + 65535) / 65536);
    bpc = bpc < 1 ? 1 : (bpc > 256 ? 256 : bpc);
    for (int32_t t = 0; t < rounds; ++t) {
        hipLaunchKernelGGL(k_fps_round, dim3(bpc, B), dim3(kFpsBlock), 0, s, t, X, w.grid.gp, w.grid.cell_start,
                           w.grid.xs, w.mind, w.brick, w.row, w.slab, w.state, n_lm_d, w.l_off, idx, radius);
    }
    return hipGetLastError();
}

}  // namespace flood
