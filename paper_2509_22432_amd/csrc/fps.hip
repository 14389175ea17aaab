// Farthest-point landmark selection on the GPU (greedy k-centre; the paper
// selects landmarks this way, Sec. 2 and Table 1).
//
// Every point keeps its running minimum squared distance to the landmarks
// chosen so far; the next landmark is the argmax of the 64-bit key
// (minimum bits << 32 | ~point index), so ties go to the lowest index.
//
// * Large clouds: one cooperative launch per cloud.  The points are sorted
//   in Morton order and cut into chunks of 64*m; chunk c belongs to
//   workgroup c mod W, which keeps the chunk's bounding box, max key and
//   argmax point in LDS.  A round updates only the chunks whose box lies
//   closer to the new landmark than the chunk's max minimum (a point
//   farther away cannot change), re-reduces the workgroup's max, publishes
//   it to a two-slot ring in global memory and polls the W slots of the
//   round: the ring replaces a grid barrier and a second reduction.  Only
//   the 64-bit keys cross workgroups (the winner's coordinates are read
//   from X), so no release/acquire fence and no L2 write-back is needed.
// * Small clouds (batches): one persistent workgroup per cloud over a
//   row-major grid.  State per row of cells and per z-slab of rows; a
//   round updates the points in the cells within the covering radius R of
//   the newest landmark (every running minimum is <= R^2), rebuilds the
//   keys of the touched rows and slabs (slab keys live in LDS) and takes
//   the argmax over the slabs.  Round 0 runs as three dense launches.
#include <algorithm>

#include "internal.hpp"

namespace flood {

static constexpr int kDenseBlock = 256;
static constexpr int kPT = 1024;       // persistent workgroup
static constexpr int kU = 8;           // points per thread per step
static constexpr int kMaxDim = 1024;   // cells per axis of a row grid (slab keys fit in LDS)
static constexpr int kMaxWG = 256;     // workgroups of one cooperative launch (ring slots per round)

struct FpsState {
    int32_t cur;  // local index of the newest landmark
    float r2;     // current max of the running minima (covering radius squared)
    float lx, ly, lz;
    int32_t pad;
};

struct FpsWork {
    GridWork grid;
    float *mind;      // [sum N] running minima, cell-sorted order
    uint64_t *rkey;   // [total cells] row keys, at the row's first cell
    FpsState *state;  // [B]
    int64_t *l_off;   // [B+1]
};

static float fps_alpha() { return 1.0f; }

size_t fps_workspace(int32_t B, const int64_t *x_off, const int32_t *n_lm) {
    (void)n_lm;
    int64_t tc = 0;
    size_t bytes = grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    bytes += sizeof(float) * np + 256;
    bytes += sizeof(uint64_t) * (tc + 1) + 256;
    bytes += sizeof(FpsState) * B + 256;
    bytes += sizeof(int64_t) * (B + 1) + 256;
    bytes += sizeof(uint64_t) * 2 * kMaxWG + 256;  // cooperative ring
    bytes += sizeof(uint32_t) + 256;
    return bytes + 1024;
}

// recipe of the landmark rule: every operation rounded to float32, no FMA
__device__ __forceinline__ float fps_d2(float px, float py, float pz, float lx, float ly, float lz) {
    const float dx = __fsub_rn(px, lx);
    const float dy = __fsub_rn(py, ly);
    const float dz = __fsub_rn(pz, lz);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

__device__ __forceinline__ uint64_t fps_key(float m, uint32_t local_idx) {
    return ((uint64_t)__float_as_uint(m) << 32) | (uint64_t)(0xffffffffu - local_idx);
}

// correctly rounded float sqrt: the double root is within one double ulp
// and the root of a float never lies that close to a float midpoint
__device__ __forceinline__ float sqrt_rn(float x) { return (float)sqrt((double)x); }

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ void finish_round(int32_t t, int32_t nl, uint64_t k, int64_t o, int64_t pt_base,
                                             const float *__restrict__ X, int32_t *__restrict__ idx_out,
                                             float *__restrict__ radius, float &lx, float &ly, float &lz,
                                             float &r2) {
    const float best = __uint_as_float((uint32_t)(k >> 32));
    const int32_t nxt = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
    if (radius) radius[o + t] = sqrt_rn(best);
    if (t + 1 < nl) idx_out[o + t + 1] = nxt;
    const int64_t row = pt_base + nxt;
    lx = X[3 * row];
    ly = X[3 * row + 1];
    lz = X[3 * row + 2];
    r2 = best;
}

__global__ void k_fps_init(int32_t B, const int32_t *n_lm, const int64_t *start, const float *X, const int64_t *x_off,
                           FpsState *st, int64_t *l_off, int32_t *idx) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t o = 0;
    for (int32_t b = 0; b < B; ++b) {
        l_off[b] = o;
        FpsState S;
        S.cur = start ? (int32_t)start[b] : 0;
        const int64_t row = x_off[b] + S.cur;
        S.lx = X[3 * row];
        S.ly = X[3 * row + 1];
        S.lz = X[3 * row + 2];
        S.r2 = INFINITY;
        S.pad = 0;
        st[b] = S;
        idx[o] = S.cur;
        o += n_lm[b];
    }
    l_off[B] = o;
}

// ---------------------------------------------------------------------------
// dense rounds

__global__ __launch_bounds__(kDenseBlock) void k_fps_dense_pts(int32_t t, const GridParam *__restrict__ gp,
                                                               const float4 *__restrict__ xs, float *__restrict__ mind,
                                                               const FpsState *__restrict__ st,
                                                               const int32_t *__restrict__ n_lm) {
    const int b = blockIdx.y;
    if (t >= n_lm[b]) return;
    const GridParam g = gp[b];
    if (g.morton) return;
    const FpsState S = st[b];
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < g.npts; p += (int64_t)gridDim.x * blockDim.x) {
        const float4 q = xs[g.pt_base + p];
        const float d2 = fps_d2(q.x, q.y, q.z, S.lx, S.ly, S.lz);
        if (d2 < mind[g.pt_base + p]) mind[g.pt_base + p] = d2;
    }
}

// one wave per row of cells: the row key over the row's points
__global__ __launch_bounds__(256) void k_fps_dense_rows(int32_t t, const GridParam *__restrict__ gp,
                                                        const uint32_t *__restrict__ cs, const float4 *__restrict__ xs,
                                                        const float *__restrict__ mind, uint64_t *__restrict__ rkey,
                                                        const int32_t *__restrict__ n_lm) {
    const int b = blockIdx.y;
    if (t >= n_lm[b]) return;
    const GridParam g = gp[b];
    if (g.morton) return;
    const int lane = threadIdx.x & 63;
    const int64_t nrows = (int64_t)g.ny * g.nz;
    const uint32_t base_idx = (uint32_t)g.pt_base;
    for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < nrows; row += (int64_t)gridDim.x * 4) {
        const int64_t c0 = g.cell_base + row * g.nx;
        const uint32_t p0 = cs[c0], p1 = cs[c0 + g.nx];
        uint64_t k = 0;
        for (uint32_t p = p0 + lane; p < p1; p += 64) {
            const uint64_t kk = fps_key(mind[p], (uint32_t)__float_as_int(xs[p].w) - base_idx);
            k = kk > k ? kk : k;
        }
        k = wave_max_u64(k);
        if (lane == 0) rkey[c0] = k;
    }
}

__global__ __launch_bounds__(kPT) void k_fps_dense_argmax(int32_t t, const float *__restrict__ X,
                                                          const GridParam *__restrict__ gp,
                                                          const uint64_t *__restrict__ rkey, FpsState *__restrict__ st,
                                                          const int32_t *__restrict__ n_lm,
                                                          const int64_t *__restrict__ l_off,
                                                          int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    const int b = blockIdx.x;
    if (t >= n_lm[b]) return;
    const GridParam g = gp[b];
    if (g.morton) return;
    const int64_t nrows = (int64_t)g.ny * g.nz;
    uint64_t k = 0;
    for (int64_t row = threadIdx.x; row < nrows; row += blockDim.x) {
        const uint64_t v = rkey[g.cell_base + row * g.nx];
        k = v > k ? v : k;
    }
    k = wave_max_u64(k);
    __shared__ uint64_t s_k[kPT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_k[wid] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kPT / 64; ++w) k = s_k[w] > k ? s_k[w] : k;
        float lx, ly, lz, r2;
        finish_round(t, n_lm[b], k, l_off[b], g.pt_base, X, idx_out, radius, lx, ly, lz, r2);
        st[b].cur = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
        st[b].r2 = r2;
        st[b].lx = lx;
        st[b].ly = ly;
        st[b].lz = lz;
    }
}

// ---------------------------------------------------------------------------
// persistent rounds

__device__ inline uint32_t block_scan_u32(uint32_t v, uint32_t *total, uint32_t *s_w) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const uint32_t w = lane < kPT / 64 ? s_w[lane] : 0u;
        uint32_t z = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(z, o, 64);
            if (lane >= o) z += y;
        }
        if (lane < kPT / 64) s_w[lane] = z - w;
        if (lane == kPT / 64 - 1) s_w[kPT / 64] = z;
    }
    __syncthreads();
    const uint32_t r = s_w[wid] + x - v;
    *total = s_w[kPT / 64];
    __syncthreads();
    return r;
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// row rr of the flattened list holding item kk (s_off: exclusive offsets, s_off[nr] = total)
__device__ __forceinline__ int find_row(const uint32_t *s_off, int nr, uint32_t k0) {
    int rr = 0, hi_r = nr;  // s_off[rr] <= k0 < s_off[hi_r]
    while (hi_r - rr > 1) {
        const int mid = (rr + hi_r) >> 1;
        if (s_off[mid] <= k0) rr = mid;
        else hi_r = mid;
    }
    return rr;
}

__global__ __launch_bounds__(kPT) void k_fps_persist(
    int32_t t0, const float *__restrict__ X, const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs,
    const float4 *__restrict__ xs, float *__restrict__ mind, uint64_t *__restrict__ rkey,
    const FpsState *__restrict__ st, const int32_t *__restrict__ n_lm, const int64_t *__restrict__ l_off,
    int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    const int b = blockIdx.x;
    const int nl = n_lm[b];
    if (t0 >= nl) return;
    const GridParam g = gp[b];
    if (g.morton) return;
    __shared__ uint64_t s_slab[kMaxDim];
    __shared__ uint64_t s_row[kPT];
    __shared__ uint32_t s_pa[kPT], s_off[kPT + 1], s_w[kPT / 64 + 1];
    __shared__ uint64_t s_rk[kPT / 64];
    __shared__ float s_l[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t slab_cells = (int64_t)g.ny * g.nx;
    for (int z = tid; z < g.nz; z += kPT) s_slab[z] = 0ull;
    if (tid == 0) {
        const FpsState S = st[b];
        s_l[0] = S.lx;
        s_l[1] = S.ly;
        s_l[2] = S.lz;
        s_l[3] = S.r2;
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)g.ny * g.nz; e += kPT) {
        const uint64_t v = rkey[g.cell_base + e * g.nx];
        if (v) atomicMax((unsigned long long *)&s_slab[e / g.ny], (unsigned long long)v);
    }
    __syncthreads();
    const uint32_t base_idx = (uint32_t)g.pt_base;
    const int64_t o = l_off[b];
    const int n[3] = {g.nx, g.ny, g.nz};
    const float og[3] = {g.ox, g.oy, g.oz};
    for (int t = t0; t < nl; ++t) {
        const float lx = s_l[0], ly = s_l[1], lz = s_l[2], r2 = s_l[3];
        const float l[3] = {lx, ly, lz};
        int lo[3], hi[3];
        const float R = sqrtf(r2);
        for (int a = 0; a < 3; ++a) {
            // one cell of margin keeps the box conservative under rounding
            const float tl = fminf(fmaxf((l[a] - R - og[a]) * g.inv_h, -4.f), (float)n[a] + 4.f);
            const float th = fminf(fmaxf((l[a] + R - og[a]) * g.inv_h, -4.f), (float)n[a] + 4.f);
            lo[a] = clampi((int)floorf(tl) - 1, 0, n[a] - 1);
            hi[a] = clampi((int)floorf(th) + 1, 0, n[a] - 1);
        }
        const int nyb = hi[1] - lo[1] + 1;
        const int nrows = nyb * (hi[2] - lo[2] + 1);
        for (int c0 = 0; c0 < nrows; c0 += kPT) {
            const int nr = min(kPT, nrows - c0);
            int64_t rowcell = 0;
            uint32_t cnt = 0, ra = 0, rlen = 0;
            if (tid < nr) {
                const int r = c0 + tid;
                const int z = lo[2] + r / nyb, y = lo[1] + r % nyb;
                rowcell = g.cell_base + ((int64_t)z * g.ny + y) * g.nx;
                ra = cs[rowcell];
                const uint32_t pa = cs[rowcell + lo[0]];
                cnt = cs[rowcell + hi[0] + 1] - pa;
                rlen = cs[rowcell + g.nx] - ra;
                s_pa[tid] = pa;
                s_row[tid] = 0ull;
            }
            // (a) minima of the box's points
            uint32_t total;
            uint32_t off = block_scan_u32(cnt, &total, s_w);
            s_off[tid] = off;
            if (tid == kPT - 1) s_off[kPT] = total;
            __syncthreads();
            for (uint32_t k0 = (uint32_t)tid * kU; k0 < total; k0 += kPT * kU) {
                int rr = find_row(s_off, nr, k0);
                uint32_t pp[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const uint32_t kk = k0 + u;
                    pp[u] = 0xffffffffu;
                    if (kk < total) {
                        while (s_off[rr + 1] <= kk) ++rr;
                        pp[u] = s_pa[rr] + (kk - s_off[rr]);
                    }
                }
                float4 qq[kU];
                float mm[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    if (pp[u] != 0xffffffffu) {
                        qq[u] = xs[pp[u]];
                        mm[u] = mind[pp[u]];
                    }
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    if (pp[u] != 0xffffffffu) {
                        const float d2 = fps_d2(qq[u].x, qq[u].y, qq[u].z, lx, ly, lz);
                        if (d2 < mm[u]) mind[pp[u]] = d2;
                    }
            }
            __threadfence_block();
            __syncthreads();
            // (b) keys of the touched rows, over all their points
            if (tid < nr) s_pa[tid] = ra;
            off = block_scan_u32(rlen, &total, s_w);
            s_off[tid] = off;
            if (tid == kPT - 1) s_off[kPT] = total;
            __syncthreads();
            for (uint32_t k0 = (uint32_t)tid * kU; k0 < total; k0 += kPT * kU) {
                int rr = find_row(s_off, nr, k0);
                int rrs[kU];
                uint32_t pp[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const uint32_t kk = k0 + u;
                    pp[u] = 0xffffffffu;
                    rrs[u] = rr;
                    if (kk < total) {
                        while (s_off[rr + 1] <= kk) ++rr;
                        pp[u] = s_pa[rr] + (kk - s_off[rr]);
                        rrs[u] = rr;
                    }
                }
                float mm[kU];
                uint32_t ii[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    if (pp[u] != 0xffffffffu) {
                        mm[u] = mind[pp[u]];
                        ii[u] = (uint32_t)__float_as_int(xs[pp[u]].w) - base_idx;
                    }
                uint64_t run = 0;
                int run_row = rrs[0];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (pp[u] == 0xffffffffu) continue;
                    if (rrs[u] != run_row) {
                        if (run) atomicMax((unsigned long long *)&s_row[run_row], (unsigned long long)run);
                        run = 0;
                        run_row = rrs[u];
                    }
                    const uint64_t kk2 = fps_key(mm[u], ii[u]);
                    run = kk2 > run ? kk2 : run;
                }
                if (run) atomicMax((unsigned long long *)&s_row[run_row], (unsigned long long)run);
            }
            __syncthreads();
            if (tid < nr) rkey[rowcell] = s_row[tid];
            __threadfence_block();
            __syncthreads();
        }
        // (c) touched slabs, then the argmax over all slabs
        for (int z = lo[2] + tid; z <= hi[2]; z += kPT) s_slab[z] = 0ull;
        __syncthreads();
        const int nzt = hi[2] - lo[2] + 1;
        for (int e0 = tid * 4; e0 < nzt * g.ny; e0 += kPT * 4) {
            uint64_t vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u;
                vv[u] = 0;
                if (e < nzt * g.ny)
                    vv[u] = rkey[g.cell_base + (int64_t)(lo[2] + e / g.ny) * slab_cells + (int64_t)(e % g.ny) * g.nx];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (vv[u]) atomicMax((unsigned long long *)&s_slab[lo[2] + (e0 + u) / g.ny], (unsigned long long)vv[u]);
        }
        __syncthreads();
        uint64_t k = 0;
        for (int z = tid; z < g.nz; z += kPT) k = s_slab[z] > k ? s_slab[z] : k;
        k = wave_max_u64(k);
        if (lane == 0) s_rk[wid] = k;
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kPT / 64; ++w) k = s_rk[w] > k ? s_rk[w] : k;
            float nlx, nly, nlz, nr2;
            finish_round(t, nl, k, o, g.pt_base, X, idx_out, radius, nlx, nly, nlz, nr2);
            s_l[0] = nlx;
            s_l[1] = nly;
            s_l[2] = nlz;
            s_l[3] = nr2;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// cooperative rounds (large clouds)

static constexpr int kMaxCpw = 4096;              // chunk slots per workgroup (36 B of LDS each)
static constexpr int64_t kCoopMin = 1 << 19;      // clouds of at least this many points
static constexpr int64_t kCoopMaxPts = 1 << 30;   // the ring key keeps 30 index bits
static constexpr int kSpinLimit = 1 << 22;        // polls of one round before the launch gives up

struct CoopArgs {
    int32_t b;       // cloud
    int32_t nl;      // landmarks
    int32_t nwg;     // working workgroups W
    int32_t pad;
    int64_t nchunk;  // chunks of 64*m points
    int64_t lo;      // first landmark slot of the cloud in idx/radius
};

// lower bound of fps_d2 over a box, with the same operations: each rounded
// operation is monotone, so no point of the box can score below it
__device__ __forceinline__ float fps_box_d2(float lx, float ly, float lz, const float *bb) {
    const float dx = lx < bb[0] ? __fsub_rn(bb[0], lx) : (lx > bb[3] ? __fsub_rn(lx, bb[3]) : 0.f);
    const float dy = ly < bb[1] ? __fsub_rn(bb[1], ly) : (ly > bb[4] ? __fsub_rn(ly, bb[4]) : 0.f);
    const float dz = lz < bb[2] ? __fsub_rn(bb[2], lz) : (lz > bb[5] ? __fsub_rn(lz, bb[5]) : 0.f);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// ring key: minimum bits << 32 | tag << 30 | (2^30 - 1 - index); the 2-bit
// tag (round + 1) mod 4 tells a slot written this round from one written
// two rounds ago or cleared before the launch
__device__ __forceinline__ uint64_t ring_key(uint64_t k, uint32_t tag) {
    const uint32_t idx = 0xffffffffu - (uint32_t)k;
    return (k & 0xffffffff00000000ull) | ((uint64_t)tag << 30) | (uint64_t)(0x3fffffffu - idx);
}

// LM = log2(m) points per lane per chunk.  Keys cross workgroups through
// memory (agent-scope atomics: each XCD has its own L2); a stale slot never
// carries the round's tag, so it only delays the poll.
// LDS per chunk slot: max key, box (6 floats), list entry.
template <int LM>
__global__ __launch_bounds__(256) void k_fps_coop(
    CoopArgs a, const float *__restrict__ X, const GridParam *__restrict__ gp, const float4 *__restrict__ xs,
    float *__restrict__ mind, uint64_t *__restrict__ rk, uint32_t *__restrict__ ctl,
    const int64_t *__restrict__ start, int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    constexpr int NT = 256;
    constexpr int NW = NT / 64;
    constexpr int M = 1 << LM;     // points per lane per chunk
    constexpr int U = 8 >> LM;     // chunks per wave step
    constexpr int PER = kMaxWG / 64;  // ring slots polled per lane
    constexpr int SCOPE = __HIP_MEMORY_SCOPE_AGENT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float s_l[4];
    __shared__ uint32_t s_n;
    __shared__ int s_abort;
    __shared__ uint64_t s_wk[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int W = a.nwg;
    const int wg = blockIdx.x;
    uint32_t *err = &ctl[0];
    const int nmine = (int)((a.nchunk - wg + W - 1) / W);  // chunk slots owned (W <= nchunk)
    uint64_t *s_key = (uint64_t *)smem;
    float *s_bb = (float *)(s_key + nmine);
    uint32_t *s_list = (uint32_t *)(s_bb + 6 * nmine);

    const GridParam g = gp[a.b];
    const int64_t pb = g.pt_base, npts = g.npts;
    const uint32_t base_idx = (uint32_t)pb;
    if (tid == 0) {
        const int64_t row = pb + (start ? start[a.b] : 0);
        s_l[0] = X[3 * row];
        s_l[1] = X[3 * row + 1];
        s_l[2] = X[3 * row + 2];
        s_abort = 0;
    }
    __syncthreads();

    for (int t = 0; t < a.nl; ++t) {
        const float lx = s_l[0], ly = s_l[1], lz = s_l[2];
        const bool init = t == 0;
        // chunks the landmark can lower (all of them in round 0)
        int naff;
        if (init) {
            naff = nmine;
        } else {
            if (tid == 0) s_n = 0;
            __syncthreads();
            for (int s0 = 0; s0 < nmine; s0 += NT) {
                const int sl = s0 + tid;
                bool hit = false;
                if (sl < nmine) {
                    const float bb[6] = {s_bb[sl], s_bb[nmine + sl], s_bb[2 * nmine + sl],
                                         s_bb[3 * nmine + sl], s_bb[4 * nmine + sl], s_bb[5 * nmine + sl]};
                    hit = fps_box_d2(lx, ly, lz, bb) < __uint_as_float((uint32_t)(s_key[sl] >> 32));
                }
                const uint64_t mask = __ballot(hit);
                uint32_t basep = 0;
                if (lane == 0 && mask) basep = atomicAdd(&s_n, (uint32_t)__popcll(mask));
                basep = __shfl(basep, 0, 64);
                if (hit) s_list[basep + __popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)sl;
            }
            __syncthreads();
            naff = (int)s_n;
        }
        // update the chunks, U per wave step with 8 loads in flight per lane
        for (int e0 = wid * U; e0 < naff; e0 += NW * U) {
            float4 q[8];
            float mm[8];
            int64_t pp[8];
            int sl[U];
#pragma unroll
            for (int c = 0; c < U; ++c) {
                const int e = e0 + c;
                sl[c] = e < naff ? (init ? e : (int)s_list[e]) : -1;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int c = i >> LM, u = i & (M - 1);
                pp[i] = -1;
                if (sl[c] >= 0) {
                    const int64_t ch = wg + (int64_t)sl[c] * W;
                    const int64_t p = (ch << (6 + LM)) + (u << 6) + lane;
                    if (p < npts) pp[i] = pb + p;
                }
                if (pp[i] >= 0) {
                    q[i] = xs[pp[i]];
                    mm[i] = init ? INFINITY : mind[pp[i]];
                }
            }
#pragma unroll
            for (int c = 0; c < U; ++c) {
                if (sl[c] < 0) continue;
                uint64_t kb = 0;
                float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY, mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY;
#pragma unroll
                for (int u = 0; u < M; ++u) {
                    const int i = c * M + u;
                    if (pp[i] < 0) continue;
                    const float d2 = fps_d2(q[i].x, q[i].y, q[i].z, lx, ly, lz);
                    if (d2 < mm[i]) {
                        mm[i] = d2;
                        mind[pp[i]] = d2;
                    }
                    const uint64_t k = fps_key(mm[i], (uint32_t)__float_as_int(q[i].w) - base_idx);
                    kb = k > kb ? k : kb;
                    if (init) {
                        mn0 = fminf(mn0, q[i].x); mx0 = fmaxf(mx0, q[i].x);
                        mn1 = fminf(mn1, q[i].y); mx1 = fmaxf(mx1, q[i].y);
                        mn2 = fminf(mn2, q[i].z); mx2 = fmaxf(mx2, q[i].z);
                    }
                }
                const uint64_t km = wave_max_u64(kb);
                if (init) {
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) {
                        mn0 = fminf(mn0, __shfl_xor(mn0, o, 64)); mx0 = fmaxf(mx0, __shfl_xor(mx0, o, 64));
                        mn1 = fminf(mn1, __shfl_xor(mn1, o, 64)); mx1 = fmaxf(mx1, __shfl_xor(mx1, o, 64));
                        mn2 = fminf(mn2, __shfl_xor(mn2, o, 64)); mx2 = fmaxf(mx2, __shfl_xor(mx2, o, 64));
                    }
                }
                if (lane == 0) {
                    const int s_ = sl[c];
                    s_key[s_] = km;
                    if (init) {
                        s_bb[s_] = mn0; s_bb[nmine + s_] = mn1; s_bb[2 * nmine + s_] = mn2;
                        s_bb[3 * nmine + s_] = mx0; s_bb[4 * nmine + s_] = mx1; s_bb[5 * nmine + s_] = mx2;
                    }
                }
            }
        }
        __syncthreads();
        // the workgroup's max key
        uint64_t kb = 0;
        for (int sl = tid; sl < nmine; sl += NT) kb = s_key[sl] > kb ? s_key[sl] : kb;
        const uint64_t km = wave_max_u64(kb);
        if (lane == 0) s_wk[wid] = km;
        __syncthreads();
        if (wid == 0) {
            const uint32_t tag = (uint32_t)(t + 1) & 3u;
            uint64_t *ring = rk + (t & 1) * kMaxWG;
            if (lane == 0) {
                uint64_t k = s_wk[0];
                for (int w = 1; w < NW; ++w) k = s_wk[w] > k ? s_wk[w] : k;
                __hip_atomic_store(&ring[wg], ring_key(k, tag), __ATOMIC_RELAXED, SCOPE);
            }
            // poll the round's W slots; each slot's point is fetched from X as
            // soon as its key shows up, so the winner's is usually on hand
            uint64_t v[PER];
            float cx[PER], cy[PER], cz[PER];
            bool have[PER];
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                v[i] = 0;
                cx[i] = cy[i] = cz[i] = 0.f;
                have[i] = lane + 64 * i >= W;
            }
            bool done = false;
            for (int spin = 0; spin < kSpinLimit; ++spin) {
                bool ok = true;
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    if (have[i]) continue;
                    const uint64_t x = __hip_atomic_load(&ring[lane + 64 * i], __ATOMIC_RELAXED, SCOPE);
                    if ((((uint32_t)x >> 30) & 3u) == tag) {
                        have[i] = true;
                        v[i] = x;
                        const int64_t row = pb + (int64_t)(0x3fffffffu - ((uint32_t)x & 0x3fffffffu));
                        cx[i] = X[3 * row];
                        cy[i] = X[3 * row + 1];
                        cz[i] = X[3 * row + 2];
                    } else {
                        ok = false;
                    }
                }
                if (__all(ok)) {
                    done = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            uint64_t mk = 0;
            float bx = 0.f, by = 0.f, bz = 0.f;
#pragma unroll
            for (int i = 0; i < PER; ++i)
                if (v[i] > mk) {
                    mk = v[i];
                    bx = cx[i];
                    by = cy[i];
                    bz = cz[i];
                }
            const uint64_t best = wave_max_u64(mk);
            const uint64_t own = __ballot(mk == best);
            const int src = __ffsll((unsigned long long)own) - 1;
            bx = __shfl(bx, src, 64);
            by = __shfl(by, src, 64);
            bz = __shfl(bz, src, 64);
            if (lane == 0) {
                if (!done) {
                    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                    if (wg == 0)
                        for (int tt = t + 1; tt < a.nl; ++tt) idx_out[a.lo + tt] = -1;
                } else {
                    s_l[0] = bx;
                    s_l[1] = by;
                    s_l[2] = bz;
                    if (wg == 0) {
                        if (radius) radius[a.lo + t] = sqrt_rn(__uint_as_float((uint32_t)(best >> 32)));
                        if (t + 1 < a.nl) idx_out[a.lo + t + 1] = (int32_t)(0x3fffffffu - ((uint32_t)best & 0x3fffffffu));
                    }
                }
            }
        }
        __syncthreads();
        if (s_abort) return;
    }
}

template <int LM>
static hipError_t launch_coop(const CoopArgs &a, int grid, int shmem, const float *X, const GridParam *gp,
                              const float4 *xs, float *mind, uint64_t *rk, uint32_t *ctl, const int64_t *start,
                              int32_t *idx, float *radius, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)k_fps_coop<LM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, shmem);
    if (e != hipSuccess) return e;
    CoopArgs aa = a;
    void *args[] = {&aa, (void *)&X, (void *)&gp, (void *)&xs, &mind, &rk, &ctl, (void *)&start, &idx, &radius};
    return hipLaunchCooperativeKernel((const void *)k_fps_coop<LM>, dim3(grid), dim3(256),
                                      args, (unsigned)shmem, s);
}

static int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

struct CoopShape {
    int32_t nwg;   // workgroups
    int lm;
    int64_t nchunk;
    int shmem;
};

// the cooperative launch of a cloud of n points (one workgroup per CU, at
// least 16 chunks each); false: the persistent path
static bool coop_shape(int64_t n, int cus, CoopShape *cs) {
    if (n < kCoopMin || n >= kCoopMaxPts || cus < 1) return false;
    const int64_t wmax = std::min<int64_t>(cus, kMaxWG);
    for (int l = 0; l <= 3; ++l) {
        const int64_t nc = (n + (64 << l) - 1) / (64 << l);
        const int64_t w = std::min<int64_t>(wmax, std::max<int64_t>(1, nc / 16));
        const int64_t cpw = (nc + w - 1) / w;
        if (cpw <= kMaxCpw) {
            cs->nwg = (int32_t)w;
            cs->lm = l;
            cs->nchunk = nc;
            cs->shmem = (int)(cpw * 36);
            return true;
        }
    }
    return false;
}

// clouds below this size (and at least kCoopMin) take a cooperative path
static int64_t coop_limit(int cus) {
    const int64_t wmax = std::min<int64_t>(cus, kMaxWG);
    return std::min<int64_t>(kCoopMaxPts, wmax * kMaxCpw * 512);
}

hipError_t fps_run(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                   const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                   float *radius, void *ws, size_t ws_bytes, hipStream_t s) {
    int64_t tc = 0;
    grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    Carve c(ws, ws_bytes);
    FpsWork w;
    grid_carve(c, B, x_off, tc, w.grid);
    w.mind = c.take<float>(np);
    w.rkey = c.take<uint64_t>(tc + 1);
    w.state = c.take<FpsState>(B);
    w.l_off = c.take<int64_t>(B + 1);
    uint64_t *ring_k = c.take<uint64_t>(2 * kMaxWG);
    uint32_t *ctl = c.take<uint32_t>(1);  // error flag of the cooperative launches
    if (!c.ok()) return hipErrorOutOfMemory;
    const int cus = device_cus();
    const int64_t coop_hi = coop_limit(cus);
    hipError_t e = grid_build(X, B, x_off, x_off_d, fps_alpha(), w.grid, s, kMaxDim, kCoopMin, coop_hi);
    if (e != hipSuccess) return e;
    e = fill_f32(w.mind, INFINITY, np, s);
    if (e != hipSuccess) return e;
    e = fill_u32(ctl, 0u, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fps_init, dim3(1), dim3(1), 0, s, B, n_lm_d, start_d, X, x_off_d, w.state, w.l_off, idx);
    // large clouds: one cooperative launch each
    int64_t nmax = 0, cmax = 0, lo = 0;
    int32_t rounds = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = x_off[b + 1] - x_off[b];
        CoopShape cs;
        if (n >= kCoopMin && n < coop_hi && coop_shape(n, cus, &cs)) {
            e = fill_u64(ring_k, 0ull, 2 * kMaxWG, s);
            if (e != hipSuccess) return e;
            CoopArgs a;
            a.b = b;
            a.nl = n_lm[b];
            a.nwg = cs.nwg;
            a.pad = 0;
            a.nchunk = cs.nchunk;
            a.lo = lo;
#define FLOOD_COOP(LM_) launch_coop<LM_>(a, cs.nwg, cs.shmem, X, w.grid.gp, w.grid.xs, w.mind, ring_k, ctl, start_d, idx, radius, s)
            switch (cs.lm) {
                case 0: e = FLOOD_COOP(0); break;
                case 1: e = FLOOD_COOP(1); break;
                case 2: e = FLOOD_COOP(2); break;
                default: e = FLOOD_COOP(3); break;
            }
#undef FLOOD_COOP
            if (e != hipSuccess) return e;
        } else {
            nmax = n > nmax ? n : nmax;
            const int64_t cc = cells_cap(n, fps_alpha());
            cmax = cc > cmax ? cc : cmax;
            rounds = n_lm[b] > rounds ? n_lm[b] : rounds;
        }
        lo += n_lm[b];
    }
    if (rounds == 0) return hipGetLastError();
    // the other clouds: dense rounds while a round touches most of a large
    // cloud, then one persistent workgroup per cloud
    const int32_t t0 = std::min<int32_t>(rounds, nmax > 2000000 ? 8 : 1);
    const unsigned bp = (unsigned)std::min<int64_t>(4096, (nmax + kDenseBlock * 4 - 1) / (kDenseBlock * 4));
    const unsigned br = (unsigned)std::min<int64_t>(4096, (cmax / 32 + 3) / 4 + 1);
    for (int32_t t = 0; t < t0; ++t) {
        hipLaunchKernelGGL(k_fps_dense_pts, dim3(bp, B), dim3(kDenseBlock), 0, s, t, w.grid.gp, w.grid.xs, w.mind,
                           w.state, n_lm_d);
        hipLaunchKernelGGL(k_fps_dense_rows, dim3(br, B), dim3(256), 0, s, t, w.grid.gp, w.grid.cell_start, w.grid.xs,
                           w.mind, w.rkey, n_lm_d);
        hipLaunchKernelGGL(k_fps_dense_argmax, dim3(B), dim3(kPT), 0, s, t, X, w.grid.gp, w.rkey, w.state, n_lm_d,
                           w.l_off, idx, radius);
    }
    if (t0 < rounds)
        hipLaunchKernelGGL(k_fps_persist, dim3(B), dim3(kPT), 0, s, t0, X, w.grid.gp, w.grid.cell_start, w.grid.xs,
                           w.mind, w.rkey, w.state, n_lm_d, w.l_off, idx, radius);
    return hipGetLastError();
}

}  // namespace flood
