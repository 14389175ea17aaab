// Farthest-point landmark selection on the GPU (greedy k-centre; the paper
// selects landmarks this way, Sec. 2 and Table 1).
//
// Every point keeps its running minimum squared distance to the landmarks
// chosen so far; the next landmark is the argmax of the 64-bit key
// (minimum bits << 32 | ~point index), so ties go to the lowest index.
//
// * Large clouds: one cooperative launch per cloud.  The points are sorted
//   in Morton order and cut into chunks; chunk c belongs to workgroup
//   c mod W, which keeps the chunk's bounding box, best key and point and
//   second minimum in LDS.  Landmarks are decided in exchanges of several
//   at a time: the workgroups publish their best chunks, workgroup 0
//   replays the greedy rule on them for as long as every unseen point is
//   provably below the next pick, and the picks go back to all workgroups
//   (the section "cooperative rounds" below gives the details).  Exchanged
//   words carry the exchange number, so no release/acquire fence and no
//   L2 write-back is needed.
// * Small clouds (batches): one persistent workgroup per cloud over a
//   row-major grid.  State per row of cells and per z-slab of rows; a
//   round updates the points in the cells within the covering radius R of
//   the newest landmark (every running minimum is <= R^2), rebuilds the
//   keys of the touched rows and slabs (slab keys live in LDS) and takes
//   the argmax over the slabs.  Round 0 runs as three dense launches.
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace flood {

static constexpr int kDenseBlock = 256;
static constexpr int kPT = 1024;       // persistent workgroup
static constexpr int kU = 8;           // points per thread per step
static constexpr int kMaxDim = 1024;   // cells per axis of a row grid (slab keys fit in LDS)
static constexpr int kMaxWG = 256;     // workgroups of one cooperative launch
static constexpr int kRec = 32;        // 64-bit words of a workgroup's record in an exchange
static constexpr int kDec = 192;       // 64-bit words of an exchange's decision

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
    bytes += sizeof(uint64_t) * 2 * ((size_t)kMaxWG * kRec + kDec) + 512;  // cooperative exchange records and decisions
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
//
// One launch per cloud; chunk c of 64*m Morton-consecutive points belongs
// to workgroup c mod W, which keeps per chunk in LDS: the bounding box, the
// best key (running minimum bits << 32 | ~index) with its point, and the
// second-largest running minimum.  The landmarks are decided in exchanges
// of up to kJ at a time:
//  1. every workgroup applies the landmarks of the previous exchange to
//     the chunks they can lower (box closer than the chunk's best minimum;
//     tested first against the union box of kG consecutive slots)
//     and publishes its kK best chunks (best point, its coordinates, the
//     chunk's second minimum and box) and the key of its next chunk;
//  2. workgroup 0 collects the W records; each of its waves keeps its best
//     key and the candidates above its kT-th largest minimum (which bounds
//     the rest), and one wave replays the greedy rule on the kept ones:
//     the next landmark is the best candidate after the landmarks picked
//     so far, accepted only while its key exceeds every bound on the points
//     not in view -- the next chunks' keys, the thresholds, and per
//     published chunk min(second minimum, farthest box corner from each
//     pick); the first pick is always exact (it is the global maximum);
//  3. it publishes the picks and every workgroup reads them.
// So the picks are exactly those of the one-at-a-time greedy rule, and a
// chunk update and two exchanges through memory are shared by several
// landmarks.  Exchanged words carry the exchange number, so a stale word is
// never taken for a fresh one.

static constexpr int kMaxCpw = 2560;              // chunk slots per workgroup (60 B of LDS each)
static constexpr int kG = 8;                      // consecutive chunk slots of a workgroup under one group bound
static constexpr int64_t kCoopMin = 1 << 19;      // clouds of at least this many points
static constexpr int64_t kCoopMinFew = 1 << 12;   // ... or of this many, in calls of at most kFewClouds clouds
static constexpr int32_t kFewClouds = 8;
static constexpr int kSpinLimit = 1 << 22;        // polls of one exchange before the launch gives up
static constexpr int kK = 2;                      // candidates a workgroup publishes
static constexpr int kJ = 32;                     // landmarks decided per exchange, at most
using LMask = std::conditional_t<(kJ > 32), uint64_t, uint32_t>;  // a set of an exchange's landmarks
static constexpr int kT = 16;                     // candidates each leader wave keeps for the replay

struct CoopArgs {
    int32_t b;       // cloud
    int32_t nl;      // landmarks
    int32_t nwg;     // workgroups W
    int32_t pad;
    int64_t nchunk;  // chunks of 64*m points
    int64_t lo;      // first landmark slot of the cloud in idx/radius
};

// lower bound of fps_d2 over a box, with the same operations: each rounded
// operation is monotone, so no point of the box can score below it.  Per
// axis the distance to the slab is max(lo - l, l - hi, 0): at most one of the
// two rounded differences is positive (a rounded difference keeps its sign).
__device__ __forceinline__ float slab_d(float l, float lo, float hi) {
    return fmaxf(fmaxf(__fsub_rn(lo, l), __fsub_rn(l, hi)), 0.f);
}
__device__ __forceinline__ float fps_box_d2(float lx, float ly, float lz, const float *bb) {
    const float dx = slab_d(lx, bb[0], bb[3]);
    const float dy = slab_d(ly, bb[1], bb[4]);
    const float dz = slab_d(lz, bb[2], bb[5]);
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// upper bound of fps_d2 over a box: per axis the larger rounded difference
// to the two faces (fl(p - l) is monotone in p)
__device__ __forceinline__ float fps_box_far_d2(float lx, float ly, float lz, const float *bb) {
    const float dx = fmaxf(fabsf(__fsub_rn(bb[0], lx)), fabsf(__fsub_rn(bb[3], lx)));
    const float dy = fmaxf(fabsf(__fsub_rn(bb[1], ly)), fabsf(__fsub_rn(bb[4], ly)));
    const float dz = fmaxf(fabsf(__fsub_rn(bb[2], lz)), fabsf(__fsub_rn(bb[5], lz)));
    return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// wave reductions that end in lane 63: the four in-row DPP steps leave every
// lane of a row holding its row's reduction, then the broadcasts of lane 15
// (into rows 1 and 3) and of lane 31 (into rows 2 and 3) combine the rows, so
// lane 63 holds the reduction of all 64 lanes and one scalar read fetches it
// (lanes of the rows a broadcast leaves out are never read).  All 64 lanes
// active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_max_rows(uint32_t v) {
    return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_min_rows(uint32_t v) {
    return min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, CTRL, ROWS, 0xf, true));
}
__device__ __forceinline__ uint32_t wave_max_u32_l63(uint32_t v) {
    v = dpp_max_u32<0x140>(dpp_max_u32<0x141>(dpp_max_u32<0x4e>(dpp_max_u32<0xb1>(v))));
    v = dpp_max_rows<0x143, 0xc>(dpp_max_rows<0x142, 0xa>(v));
    return rd_lane(v, 63);
}
__device__ __forceinline__ uint32_t wave_min_u32_l63(uint32_t v) {
    v = dpp_min_u32<0x140>(dpp_min_u32<0x141>(dpp_min_u32<0x4e>(dpp_min_u32<0xb1>(v))));
    v = dpp_min_rows<0x143, 0xc>(dpp_min_rows<0x142, 0xa>(v));
    return rd_lane(v, 63);
}
// the writelane intrinsic (v_writelane_b32): old with lane l replaced by the
// uniform value v
__device__ int32_t amdgcn_writelane(int32_t v, int32_t l, int32_t old) __asm("llvm.amdgcn.writelane.i32");
// the largest of non-negative floats (ordered as their bits)
__device__ __forceinline__ float wave_max_nonneg(float v) { return __uint_as_float(wave_max_u32_l63(__float_as_uint(v))); }
// the lane holding the wave's largest key (mb << 32) | ~id: the largest mb,
// and among equal mb the lowest id; mmax gets that mb
__device__ __forceinline__ int wave_argmax_key63(uint32_t mb, uint32_t id, uint32_t &mmax) {
    mmax = wave_max_u32_l63(mb);
    const uint64_t tied = __ballot(mb == mmax);
    int src = __ffsll((unsigned long long)tied) - 1;
    if (__popcll(tied) != 1) {
        const uint32_t umin = wave_min_u32_l63(mb == mmax ? id : 0xffffffffu);
        src = __ffsll((unsigned long long)__ballot(mb == mmax && id == umin)) - 1;
    }
    return src;
}

// an exchanged word: 32-bit payload, 32-bit exchange number
__device__ __forceinline__ uint64_t xw(uint32_t payload, uint32_t id) { return ((uint64_t)payload << 32) | id; }
__device__ __forceinline__ uint32_t xw_val(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ bool xw_ok(uint64_t w, uint32_t id) { return (uint32_t)w == id; }

// keep the three largest (key, slot) pairs
__device__ __forceinline__ void top3_insert(uint64_t (&k)[3], int (&s)[3], uint64_t v, int sv) {
    if (v > k[2]) {
        if (v > k[1]) {
            k[2] = k[1];
            s[2] = s[1];
            if (v > k[0]) {
                k[1] = k[0];
                s[1] = s[0];
                k[0] = v;
                s[0] = sv;
            } else {
                k[1] = v;
                s[1] = sv;
            }
        } else {
            k[2] = v;
            s[2] = sv;
        }
    }
}

__device__ __forceinline__ uint32_t uniform_mask(uint32_t m) { return __builtin_amdgcn_readfirstlane(m); }
__device__ __forceinline__ uint64_t uniform_mask(uint64_t m) {
    return (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)m) |
           ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32);
}

// threads of a cooperative workgroup: twelve waves for chunks of 64 points
// (three per SIMD: the kernel fits in 168 registers when the update takes
// four chunks per wave step), eight for larger chunks (two per SIMD)
constexpr int coop_threads(int lm) { return lm == 0 ? 768 : 512; }

template <int LM>
__global__ __launch_bounds__(coop_threads(LM)) void k_fps_coop(
    CoopArgs a, const float *__restrict__ X, const GridParam *__restrict__ gp, const float4 *__restrict__ xs,
    float *__restrict__ mind, uint64_t *__restrict__ rec, uint64_t *__restrict__ dec, uint32_t *__restrict__ ctl,
    const int64_t *__restrict__ start, int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    // the chunk tests, updates and top three spread over all the waves; the
    // records are collected by the first NWC, one workgroup per lane
    constexpr int NT = coop_threads(LM);
    constexpr int NW = NT / 64;
    constexpr int NWC = kMaxWG / 64;
    constexpr int M = 1 << LM;          // points per lane per chunk
    constexpr int U = LM == 0 ? 4 : 8 >> LM;  // chunks per wave step
    constexpr int P = U * M;            // points per lane per wave step
    constexpr int SCOPE = __HIP_MEMORY_SCOPE_AGENT;
    constexpr int DH = (1 + 5 * kJ + 63) / 64;  // decision words a lane reads
    static_assert(1 + 12 * kK <= kRec && 1 + 12 * kK <= 64 && 1 + 5 * kJ <= kDec && kDec <= 64 * DH && kK <= 2,
                  "exchange layout");
    static_assert(NWC * kT % 64 == 0 && kT <= 64 && NWC <= NW, "whole kept candidates per lane of the replaying wave");
    static_assert(kJ <= 8 * (int)sizeof(LMask), "landmark masks");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float s_pk[kJ][3];       // landmarks to apply
    __shared__ int s_np, s_j, s_abort;
    __shared__ uint32_t s_n;
    __shared__ uint64_t s_tk[NW][3];
    __shared__ int s_ts[NW][3];
    struct Cand {
        uint64_t key;                    // 0: no candidate
        float cb, x, y, z, bb[6];
    };
    __shared__ Cand s_cand[NWC * kT];    // the leader's kept candidates
    __shared__ float s_bnd[NW];          // bound of the candidates each wave did not keep
    __shared__ uint32_t s_pick[kJ][5];   // the leader's picks
    __shared__ int s_wok[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int W = a.nwg;
    const int wg = blockIdx.x;
    uint32_t *err = &ctl[0];
    const int nmine = (int)((a.nchunk - wg + W - 1) / W);  // chunk slots owned (W <= nchunk)
    const int ngrp = (nmine + kG - 1) / kG;           // groups of kG slots (slot order is Morton order)
    uint64_t *s_key = (uint64_t *)smem;
    LMask *s_lmask = (LMask *)(s_key + nmine);        // landmarks that can lower a listed chunk
    LMask *s_gmask = s_lmask + nmine;                 // landmarks that can reach a group
    float *s_bb = (float *)(s_gmask + ngrp);
    float *s_px = s_bb + 6 * nmine;
    float *s_sec = s_px + 3 * nmine;
    uint32_t *s_list = (uint32_t *)(s_sec + nmine);  // listed chunk slots
    float *s_gbb = (float *)(s_list + nmine);         // group boxes (union of the slot boxes)
    float *s_gkm = s_gbb + 6 * ngrp;                  // group best minima (largest slot minimum)

    const GridParam g = gp[a.b];
    const int64_t pb = g.pt_base, npts = g.npts;
    const uint32_t base_idx = (uint32_t)pb;
    if (tid == 0) {
        const int64_t row = pb + (start ? start[a.b] : 0);
        s_pk[0][0] = X[3 * row];
        s_pk[0][1] = X[3 * row + 1];
        s_pk[0][2] = X[3 * row + 2];
        s_np = 1;
        s_abort = 0;
    }
    __syncthreads();

    int t_done = 1;  // landmark slots decided (slot 0 is the start point)
    for (uint32_t e = 0;; ++e) {
        const bool init = e == 0;
        const int np = s_np;
        // landmark t of this exchange in lane t of every wave (for reads by
        // a uniform lane index: no LDS round trip per landmark)
        const float pk_lx = lane < np ? s_pk[lane][0] : 0.f;
        const float pk_ly = lane < np ? s_pk[lane][1] : 0.f;
        const float pk_lz = lane < np ? s_pk[lane][2] : 0.f;
        // 1. the chunks some landmark can lower (all of them at first)
        int naff;
        if (init) {
            naff = nmine;
        } else {
            if (tid == 0) s_n = 0;
            // a) landmarks against group bounds: a landmark whose distance
            //    bound to a group box is not below the group's best minimum
            //    cannot lower any of its chunks (a slot box lies inside the
            //    group box, and the bound only grows as the box shrinks);
            //    q threads per group split the landmarks
            const int q = max(1, NT / ngrp);
            for (int u = tid; u < ngrp * q; u += NT) {
                const int gi = u / q, r = u - gi * q;
                const float gb[6] = {s_gbb[gi], s_gbb[ngrp + gi], s_gbb[2 * ngrp + gi],
                                     s_gbb[3 * ngrp + gi], s_gbb[4 * ngrp + gi], s_gbb[5 * ngrp + gi]};
                const float gkm = s_gkm[gi];
                LMask gm = 0;
                for (int t = r; t < np; t += q)
                    gm |= (LMask)(fps_box_d2(s_pk[t][0], s_pk[t][1], s_pk[t][2], gb) < gkm ? 1u : 0u) << t;
                if (gm) atomicOr(&s_gmask[gi], gm);
            }
            __syncthreads();
            // b) the slots of reached groups against those landmarks
            for (int s0 = 0; s0 < nmine; s0 += NT) {
                const int sl = s0 + tid;
                LMask hitm = 0;  // landmarks that can lower this chunk
                const LMask gm = sl < nmine ? s_gmask[sl / kG] : (LMask)0;
                if (gm) {
                    const float bb[6] = {s_bb[sl], s_bb[nmine + sl], s_bb[2 * nmine + sl],
                                         s_bb[3 * nmine + sl], s_bb[4 * nmine + sl], s_bb[5 * nmine + sl]};
                    const float km = __uint_as_float((uint32_t)(s_key[sl] >> 32));
                    for (LMask mk = gm; mk; mk &= mk - 1u) {
                        const int t = __builtin_ctzll((unsigned long long)mk);
                        hitm |= (LMask)(fps_box_d2(s_pk[t][0], s_pk[t][1], s_pk[t][2], bb) < km ? 1u : 0u) << t;
                    }
                }
                const uint64_t mask = __ballot(hitm != 0);
                uint32_t basep = 0;
                if (lane == 0 && mask) basep = atomicAdd(&s_n, (uint32_t)__popcll(mask));
                basep = __shfl(basep, 0, 64);
                if (hitm) {
                    const uint32_t at = basep + __popcll(mask & ((1ull << lane) - 1ull));
                    s_list[at] = (uint32_t)sl;
                    s_lmask[at] = hitm;
                }
            }
            __syncthreads();
            naff = (int)s_n;
            for (int gi = tid; gi < ngrp; gi += NT) s_gmask[gi] = 0;  // read again only after later barriers
        }
        // 2. update them with the landmarks that can lower them (a landmark
        //    whose box bound is not below the chunk's best minimum leaves every
        //    running minimum of the chunk as it is): running minima, best key
        //    and point, second minimum
        for (int e0 = 0; e0 < naff; e0 += NW * U) {  // list entries e0 + c * NW + wid
            float4 q[P];
            float mm[P];
            int64_t pp[P];
            int sl[U];
            LMask msk[U];
#pragma unroll
            for (int c = 0; c < U; ++c) {
                const int ee = e0 + c * NW + wid;
                sl[c] = -1;
                msk[c] = 0;
                if (ee < naff) {
                    sl[c] = init ? ee : (int)__builtin_amdgcn_readfirstlane(s_list[ee]);
                    msk[c] = init ? (LMask)1 : uniform_mask(s_lmask[ee]);
                }
            }
#pragma unroll
            for (int i = 0; i < P; ++i) {
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
                float mb = 0.f, m2 = 0.f;  // this lane's best minimum and its second
                float bx = 0.f, by = 0.f, bz = 0.f;
                float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY, mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY;
                float d2v[M];
#pragma unroll
                for (int u = 0; u < M; ++u) d2v[u] = mm[c * M + u];
                for (LMask mk = msk[c]; mk; mk &= mk - 1u) {
                    const int t = __builtin_ctzll((unsigned long long)mk);
                    const float lx = __uint_as_float(rd_lane(__float_as_uint(pk_lx), t));
                    const float ly = __uint_as_float(rd_lane(__float_as_uint(pk_ly), t));
                    const float lz = __uint_as_float(rd_lane(__float_as_uint(pk_lz), t));
#pragma unroll
                    for (int u = 0; u < M; ++u) {
                        const int i = c * M + u;
                        if (pp[i] >= 0) d2v[u] = fminf(d2v[u], fps_d2(q[i].x, q[i].y, q[i].z, lx, ly, lz));
                    }
                }
#pragma unroll
                for (int u = 0; u < M; ++u) {
                    const int i = c * M + u;
                    if (pp[i] < 0) continue;
                    const float d2 = d2v[u];
                    if (d2 < mm[i]) {
                        mm[i] = d2;
                        mind[pp[i]] = d2;
                    }
                    const uint64_t k = fps_key(mm[i], (uint32_t)__float_as_int(q[i].w) - base_idx);
                    if (k > kb) {
                        m2 = kb ? mb : m2;
                        kb = k;
                        mb = mm[i];
                        bx = q[i].x;
                        by = q[i].y;
                        bz = q[i].z;
                    } else {
                        m2 = fmaxf(m2, mm[i]);
                    }
                    if (init) {
                        mn0 = fminf(mn0, q[i].x); mx0 = fmaxf(mx0, q[i].x);
                        mn1 = fminf(mn1, q[i].y); mx1 = fmaxf(mx1, q[i].y);
                        mn2 = fminf(mn2, q[i].z); mx2 = fmaxf(mx2, q[i].z);
                    }
                }
                uint32_t kmb;
                const int src = wave_argmax_key63((uint32_t)(kb >> 32), 0xffffffffu - (uint32_t)kb, kmb);
                const uint64_t km = ((uint64_t)kmb << 32) | rd_lane((uint32_t)kb, src);
                bx = __uint_as_float(rd_lane(__float_as_uint(bx), src));
                by = __uint_as_float(rd_lane(__float_as_uint(by), src));
                bz = __uint_as_float(rd_lane(__float_as_uint(bz), src));
                // second minimum of the chunk: every lane's best except the
                // chunk's best point, and every lane's second
                const float sec = wave_max_nonneg(lane == src ? m2 : fmaxf(mb, m2));
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
                    s_px[s_] = bx;
                    s_px[nmine + s_] = by;
                    s_px[2 * nmine + s_] = bz;
                    s_sec[s_] = sec;
                    if (init) {
                        s_bb[s_] = mn0; s_bb[nmine + s_] = mn1; s_bb[2 * nmine + s_] = mn2;
                        s_bb[3 * nmine + s_] = mx0; s_bb[4 * nmine + s_] = mx1; s_bb[5 * nmine + s_] = mx2;
                    }
                }
            }
        }
        __syncthreads();
        // group bounds: the boxes once, the best minima after every update
        for (int gi = tid; gi < ngrp; gi += NT) {
            const int s_lo = gi * kG, s_hi = min(nmine, s_lo + kG);
            float gkm = 0.f;
            for (int sl = s_lo; sl < s_hi; ++sl) gkm = fmaxf(gkm, __uint_as_float((uint32_t)(s_key[sl] >> 32)));
            s_gkm[gi] = gkm;
            if (init) {
                for (int f = 0; f < 3; ++f) {
                    float lo = INFINITY, hi = -INFINITY;
                    for (int sl = s_lo; sl < s_hi; ++sl) {
                        lo = fminf(lo, s_bb[f * nmine + sl]);
                        hi = fmaxf(hi, s_bb[(3 + f) * nmine + sl]);
                    }
                    s_gbb[f * ngrp + gi] = lo;
                    s_gbb[(3 + f) * ngrp + gi] = hi;
                }
                s_gmask[gi] = 0;
            }
        }
        // 3. this workgroup's three best chunks
        {
            uint64_t tk[3] = {0, 0, 0};
            int ts[3] = {-1, -1, -1};
            for (int sl = tid; sl < nmine; sl += NT) top3_insert(tk, ts, s_key[sl], sl);
            // the wave's three best: take the best lane head three times
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                uint32_t hb;
                const int src = wave_argmax_key63((uint32_t)(tk[0] >> 32), 0xffffffffu - (uint32_t)tk[0], hb);
                const uint64_t kw = ((uint64_t)hb << 32) | rd_lane((uint32_t)tk[0], src);
                const int sw = (int)rd_lane((uint32_t)ts[0], src);
                if (lane == 0) {
                    s_tk[wid][r] = kw;
                    s_ts[wid][r] = kw ? sw : -1;
                }
                if (lane == src) {
                    tk[0] = tk[1];
                    ts[0] = ts[1];
                    tk[1] = tk[2];
                    ts[1] = ts[2];
                    tk[2] = 0;
                    ts[2] = -1;
                }
            }
        }
        __syncthreads();
        const uint32_t id = e + 1;
        // records word-major: word f of workgroup w at rec[(q * kRec + f) * kMaxWG + w]
        // (q = exchange parity), so the leader's loads of one word are contiguous
        uint64_t *my_rec = rec + (size_t)(e & 1) * kRec * kMaxWG + wg;
        if (wid == 0) {
            // 4. the record, one word per lane: bound of the other chunks,
            //    then kK candidates of 12 words
            uint64_t tk[3] = {s_tk[0][0], s_tk[0][1], s_tk[0][2]};
            int ts[3] = {s_ts[0][0], s_ts[0][1], s_ts[0][2]};
            for (int w = 1; w < NW; ++w)
#pragma unroll
                for (int r = 0; r < 3; ++r) top3_insert(tk, ts, s_tk[w][r], s_ts[w][r]);
            uint32_t v = 0;
            if (lane == 0) {
                v = ts[kK] >= 0 ? (uint32_t)(tk[kK] >> 32) : 0u;
            } else if (lane <= 12 * kK) {
                const int c = (lane - 1) / 12, f = (lane - 1) % 12;
                const int s_ = c == 0 ? ts[0] : (c == 1 ? ts[1] : ts[2]);
                const uint64_t kc = c == 0 ? tk[0] : (c == 1 ? tk[1] : tk[2]);
                if (s_ < 0) v = f == 1 ? 0xffffffffu : 0u;  // no candidate
                else if (f == 0) v = (uint32_t)(kc >> 32);
                else if (f == 1) v = 0xffffffffu - (uint32_t)kc;
                else if (f <= 4) v = __float_as_uint(s_px[(f - 2) * nmine + s_]);
                else if (f == 5) v = __float_as_uint(s_sec[s_]);
                else v = __float_as_uint(s_bb[(f - 6) * nmine + s_]);
            }
            if (lane <= 12 * kK) __hip_atomic_store(&my_rec[(size_t)lane * kMaxWG], xw(v, id), __ATOMIC_RELAXED, SCOPE);
        }
        uint64_t *my_dec = dec + (size_t)(e & 1) * kDec;
        const int jcap = min(kJ, a.nl + 1 - t_done);
        if (wg == 0) {
            // 5. the leader: the first NWC waves collect the records, one
            //    workgroup's per lane, and keep their best candidates; then
            //    one wave replays the greedy rule on the kept ones
            if (wid < NWC) {
                const int w = wid * 64 + lane;
                float cm[kK], cxp[kK], cyp[kK], czp[kK], cb[kK], cbb[kK][6], bw = 0.f;
                uint32_t cid[kK];
                bool valid[kK];
                bool done = false;
                for (int spin = 0; spin < kSpinLimit && !done; ++spin) {
                    bool ok = true;
#pragma unroll
                    for (int c = 0; c < kK; ++c) valid[c] = false;
                    if (w < W) {
                        const uint64_t *rw = rec + (size_t)(e & 1) * kRec * kMaxWG + w;
                        const uint64_t w0 = __hip_atomic_load(&rw[0], __ATOMIC_RELAXED, SCOPE);
                        ok &= xw_ok(w0, id);
                        bw = __uint_as_float(xw_val(w0));
#pragma unroll
                        for (int c = 0; c < kK; ++c) {
                            uint32_t v[12];
#pragma unroll
                            for (int f = 0; f < 12; ++f) {
                                const uint64_t x = __hip_atomic_load(&rw[(size_t)(1 + 12 * c + f) * kMaxWG], __ATOMIC_RELAXED, SCOPE);
                                ok &= xw_ok(x, id);
                                v[f] = xw_val(x);
                            }
                            valid[c] = v[1] != 0xffffffffu;
                            cm[c] = __uint_as_float(v[0]);
                            cid[c] = v[1];
                            cxp[c] = __uint_as_float(v[2]);
                            cyp[c] = __uint_as_float(v[3]);
                            czp[c] = __uint_as_float(v[4]);
                            cb[c] = __uint_as_float(v[5]);
#pragma unroll
                            for (int f = 0; f < 6; ++f) cbb[c][f] = __uint_as_float(v[6 + f]);
                        }
                    }
                    done = __all(ok);
                    if (!done) __builtin_amdgcn_s_sleep(1);
                }
                if (lane == 0) s_wok[wid] = done ? 1 : 0;
                {
                    // every wave keeps its best key and the candidates whose
                    // minimum exceeds theta, the kT-th largest minimum it holds
                    // (found bit by bit, so at most kT - 1 lie above it); the
                    // points of every other chunk it holds have running minima of
                    // at most max(theta, the next-chunk bounds), since a chunk's
                    // second minimum never exceeds its best
                    uint64_t k[kK];
                    uint32_t mk[kK];
                    uint64_t kb = 0;
#pragma unroll
                    for (int c = 0; c < kK; ++c) {
                        const bool vc = w < W && valid[c];
                        mk[c] = vc ? __float_as_uint(cm[c]) : 0u;
                        k[c] = vc ? ((uint64_t)mk[c] << 32) | (uint64_t)(0xffffffffu - cid[c]) : 0;
                        kb = k[c] > kb ? k[c] : kb;
                    }
                    uint32_t hbest;
                    const int ksrc = wave_argmax_key63((uint32_t)(kb >> 32), 0xffffffffu - (uint32_t)kb, hbest);
                    const uint64_t ktop = ((uint64_t)hbest << 32) | rd_lane((uint32_t)kb, ksrc);
                    uint32_t th = 0;
                    for (int bit = 30; bit >= 0; --bit) {  // minima are non-negative floats
                        const uint32_t t = th | (1u << bit);
                        int cnt = 0;
#pragma unroll
                        for (int c = 0; c < kK; ++c) cnt += __popcll(__ballot(mk[c] >= t));
                        if (cnt >= kT) th = t;
                    }
                    const uint64_t below = (1ull << lane) - 1ull;
                    int base = 0;
#pragma unroll
                    for (int c = 0; c < kK; ++c) {
                        const bool in = k[c] != 0 && (mk[c] > th || k[c] == ktop);
                        const uint64_t m = __ballot(in);
                        if (in) {
                            Cand &o = s_cand[wid * kT + base + __popcll(m & below)];
                            o.key = k[c];
                            o.cb = cb[c];
                            o.x = cxp[c];
                            o.y = cyp[c];
                            o.z = czp[c];
#pragma unroll
                            for (int f = 0; f < 6; ++f) o.bb[f] = cbb[c][f];
                        }
                        base += __popcll(m);
                    }
                    if (lane >= base && lane < kT) s_cand[wid * kT + lane].key = 0;
                    const float bmax = wave_max_nonneg(w < W ? bw : 0.f);
                    if (lane == 0) s_bnd[wid] = fmaxf(bmax, __uint_as_float(th));
                }
            }
            __syncthreads();
            const bool all_in = s_wok[0] && s_wok[1] && s_wok[2] && s_wok[3];
            int j = 0;
            if (all_in && wid == 0) {
                // one wave replays the greedy rule on the NWC * kT kept
                // candidates, kR per lane.  Minima and bounds are held as the
                // bits of non-negative floats (ordered as unsigned integers);
                // an empty slot holds minimum 0, bound 0 and index ~0, so it
                // never wins against a candidate and never lowers a bound
                constexpr int kR = NWC * kT / 64;
                uint32_t m[kR], b[kR], lid[kR];
                float x[kR], y[kR], z[kR], bb[kR][6];
#pragma unroll
                for (int r = 0; r < kR; ++r) {
                    const Cand &o = s_cand[lane + 64 * r];
                    const bool alive = o.key != 0;
                    m[r] = alive ? (uint32_t)(o.key >> 32) : 0u;
                    b[r] = alive ? __float_as_uint(o.cb) : 0u;
                    lid[r] = alive ? 0xffffffffu - (uint32_t)o.key : 0xffffffffu;
                    x[r] = o.x;
                    y[r] = o.y;
                    z[r] = o.z;
#pragma unroll
                    for (int f = 0; f < 6; ++f) bb[r][f] = o.bb[f];
                }
                const uint32_t b0 = __builtin_amdgcn_readfirstlane(
                    __float_as_uint(fmaxf(fmaxf(s_bnd[0], s_bnd[1]), fmaxf(s_bnd[2], s_bnd[3]))));
                // lane p keeps pick p until the replay ends
                uint32_t pk_i = 0, pk_m = 0, pk_x = 0, pk_y = 0, pk_z = 0;
                for (int p = 0; p < jcap; ++p) {
                    // this lane's best candidate (largest minimum, then lowest index)
                    uint32_t mb = m[0], ib = lid[0], hb = b[0];
                    float bx = x[0], by = y[0], bz = z[0];
#pragma unroll
                    for (int r = 1; r < kR; ++r) {
                        if (m[r] > mb || (m[r] == mb && lid[r] < ib)) {
                            mb = m[r];
                            ib = lid[r];
                            bx = x[r];
                            by = y[r];
                            bz = z[r];
                        }
                        hb = max(hb, b[r]);
                    }
                    uint32_t mmax;
                    const int src = wave_argmax_key63(mb, ib, mmax);
                    // a key (mmax << 32 | ~index) exceeds every key whose
                    // minimum is at most a bound exactly when mmax exceeds the
                    // bound's bits
                    if (p > 0 && (!(mmax > b0) || __ballot(!(mmax > hb)))) break;
                    const uint32_t pid = rd_lane(ib, src);
                    const float px = __uint_as_float(rd_lane(__float_as_uint(bx), src));
                    const float py = __uint_as_float(rd_lane(__float_as_uint(by), src));
                    const float pz = __uint_as_float(rd_lane(__float_as_uint(bz), src));
                    pk_i = (uint32_t)amdgcn_writelane((int)pid, p, (int)pk_i);
                    pk_m = (uint32_t)amdgcn_writelane((int)mmax, p, (int)pk_m);
                    pk_x = (uint32_t)amdgcn_writelane((int)__float_as_uint(px), p, (int)pk_x);
                    pk_y = (uint32_t)amdgcn_writelane((int)__float_as_uint(py), p, (int)pk_y);
                    pk_z = (uint32_t)amdgcn_writelane((int)__float_as_uint(pz), p, (int)pk_z);
                    ++j;
                    // the candidates and their chunks' bounds after this pick
                    // (both distances are non-negative floats)
#pragma unroll
                    for (int r = 0; r < kR; ++r) {
                        m[r] = min(m[r], __float_as_uint(fps_d2(x[r], y[r], z[r], px, py, pz)));
                        b[r] = min(b[r], __float_as_uint(fps_box_far_d2(px, py, pz, bb[r])));
                    }
                }
                if (lane < j) {
                    s_pick[lane][0] = pk_i;
                    s_pick[lane][1] = pk_m;
                    s_pick[lane][2] = pk_x;
                    s_pick[lane][3] = pk_y;
                    s_pick[lane][4] = pk_z;
                }
            }
            __syncthreads();
            if (wid == 0) {
                // the decision, one word per lane: j, then 5 words per pick
                if (!all_in) {
                    if (lane == 0) {
                        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&my_dec[0], xw(0u, id), __ATOMIC_RELAXED, SCOPE);  // j = 0: abort
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < DH; ++h) {
                        const int i = lane + 64 * h;
                        if (i > 5 * j) continue;
                        const uint32_t v = i == 0 ? (uint32_t)j : s_pick[(i - 1) / 5][(i - 1) % 5];
                        __hip_atomic_store(&my_dec[i], xw(v, id), __ATOMIC_RELAXED, SCOPE);
                    }
                }
            }
        }
        // 6. every workgroup reads the decision (words lane + 64 h)
        if (wid == 0) {
            uint64_t x[DH];
            bool done = false;
            int j = 0;
            for (int spin = 0; spin < kSpinLimit; ++spin) {
#pragma unroll
                for (int h = 0; h < DH; ++h)
                    x[h] = lane + 64 * h <= 5 * kJ ? __hip_atomic_load(&my_dec[lane + 64 * h], __ATOMIC_RELAXED, SCOPE) : 0;
                const uint64_t w0 = __shfl(x[0], 0, 64);
                if (xw_ok(w0, id)) {
                    j = (int)xw_val(w0);
                    bool ok = true;
#pragma unroll
                    for (int h = 0; h < DH; ++h) {
                        const int i = lane + 64 * h;
                        ok &= !(i >= 1 && i <= 5 * j) || xw_ok(x[h], id);
                    }
                    if (__all(ok)) {
                        done = true;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0) {
                if (!done || j == 0) {
                    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                    if (wg == 0)
                        for (int tt = t_done; tt < a.nl; ++tt) idx_out[a.lo + tt] = -1;
                }
                s_j = j;
            }
            if (done && j > 0) {
                // word 1 + 5p + f of pick p: f = 0 index, 1 running minimum,
                // 2..4 coordinates; each lane stores the words it holds
#pragma unroll
                for (int h = 0; h < DH; ++h) {
                    const int i = lane + 64 * h;
                    if (i < 1 || i > 5 * j) continue;
                    const uint32_t v = xw_val(x[h]);
                    const int p = (i - 1) / 5, f = (i - 1) % 5;
                    const int slot = t_done + p;  // landmark slot this pick decides
                    if (f >= 2) {
                        if (slot < a.nl) s_pk[p][f - 2] = __uint_as_float(v);
                    } else if (wg == 0) {
                        if (f == 0) {
                            if (slot < a.nl) idx_out[a.lo + slot] = (int32_t)v;
                        } else if (radius) {
                            radius[a.lo + slot - 1] = sqrt_rn(__uint_as_float(v));
                        }
                    }
                }
                if (lane == 0) s_np = min(j, a.nl - t_done);
            }
        }
        __syncthreads();
        if (s_abort) return;
        t_done += s_j;
        if (t_done > a.nl) return;  // the last pick only gave the final covering radius
    }
}

template <int LM>
static hipError_t launch_coop(const CoopArgs &a, int grid, int shmem, const float *X, const GridParam *gp,
                              const float4 *xs, float *mind, uint64_t *rec, uint64_t *dec, uint32_t *ctl,
                              const int64_t *start, int32_t *idx, float *radius, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)k_fps_coop<LM>, hipFuncAttributeMaxDynamicSharedMemorySize, shmem);
    if (e != hipSuccess) return e;
    CoopArgs aa = a;
    void *args[] = {&aa, (void *)&X, (void *)&gp, (void *)&xs, &mind, &rec, &dec, &ctl, (void *)&start, &idx, &radius};
    return hipLaunchCooperativeKernel((const void *)k_fps_coop<LM>, dim3(grid), dim3(coop_threads(LM)), args, (unsigned)shmem, s);
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
    if (n < kCoopMinFew || cus < 1) return false;
    const int64_t wmax = std::min<int64_t>(cus, kMaxWG);
    for (int l = 0; l <= 3; ++l) {
        const int64_t nc = (n + (64 << l) - 1) / (64 << l);
        const int64_t w = std::min<int64_t>(wmax, std::max<int64_t>(1, nc / 16));
        const int64_t cpw = (nc + w - 1) / w;
        if (cpw <= kMaxCpw) {
            cs->nwg = (int32_t)w;
            cs->lm = l;
            cs->nchunk = nc;
            cs->shmem = (int)(cpw * (52 + sizeof(LMask)) + (cpw + kG - 1) / kG * (28 + sizeof(LMask)));
            return true;
        }
    }
    return false;
}

// clouds below this size (and at least the call's lower threshold) take the
// cooperative path: their chunk slots fit in LDS with m <= 8 on every
// workgroup
static int64_t coop_limit(int cus) {
    const int64_t wmax = std::min<int64_t>(cus, kMaxWG);
    return std::min<int64_t>((int64_t)1 << 31, wmax * kMaxCpw * 512);
}

hipError_t fps_run(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                   const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                   float *radius, void *ws, size_t ws_bytes, hipStream_t s) {
    int64_t tc = 0;
    grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    Carve c(ws, ws_bytes);
    FpsWork w;
    grid_carve(c, B, x_off, fps_alpha(), w.grid);
    w.mind = c.take<float>(np);
    w.rkey = c.take<uint64_t>(tc + 1);
    w.state = c.take<FpsState>(B);
    w.l_off = c.take<int64_t>(B + 1);
    uint64_t *rec = c.take<uint64_t>((size_t)2 * kMaxWG * kRec);
    uint64_t *dec = c.take<uint64_t>((size_t)2 * kDec);
    uint32_t *ctl = c.take<uint32_t>(1);  // error flag of the cooperative launches
    if (!c.ok()) return hipErrorOutOfMemory;
    const int cus = device_cus();
    const int64_t coop_hi = coop_limit(cus);
    // a cloud takes the cooperative launch (all CUs, one cloud at a time)
    // from kCoopMin points on; in a call of a few clouds already from
    // kCoopMinFew on, where one workgroup per cloud would leave the GPU idle
    const int64_t coop_lo = B <= kFewClouds ? kCoopMinFew : kCoopMin;
    hipError_t e = grid_build(X, B, x_off, x_off_d, fps_alpha(), w.grid, s, kMaxDim, coop_lo, coop_hi);
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
        if (n >= coop_lo && n < coop_hi && coop_shape(n, cus, &cs)) {
            e = fill_u64(rec, 0ull, (int64_t)2 * kMaxWG * kRec, s);
            if (e != hipSuccess) return e;
            e = fill_u64(dec, 0ull, 2 * kDec, s);
            if (e != hipSuccess) return e;
            CoopArgs a;
            a.b = b;
            a.nl = n_lm[b];
            a.nwg = cs.nwg;
            a.pad = 0;
            a.nchunk = cs.nchunk;
            a.lo = lo;
#define FLOOD_COOP(LM_) launch_coop<LM_>(a, cs.nwg, cs.shmem, X, w.grid.gp, w.grid.xs, w.mind, rec, dec, ctl, start_d, idx, radius, s)
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
