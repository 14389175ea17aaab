// Farthest-point landmark selection on the GPU (greedy k-centre; the paper
// selects landmarks this way, Sec. 2 and Table 1).
//
// State: the running minimum of every point (in cell-sorted order) and, per
// chunk of 2^shift consecutive sorted points, the chunk's max key
// (minimum bits << 32 | ~point index) and the position of that point.  The
// packed key makes ties go to the lowest point index.
//
// * Dense rounds (the first few rounds of a large cloud touch most points):
//   one block per chunk updates every point and its chunk key; the last
//   block of the cloud (atomic counter) takes the argmax over chunk keys.
// * Persistent rounds: one workgroup per cloud keeps all chunk keys in LDS.
//   A round updates only points in the cells within the covering radius R of
//   the newest landmark (every minimum is <= R^2, so no farther point can
//   change), flags the chunks whose argmax point was lowered, recomputes just
//   those, and takes the argmax over the LDS keys -- no launch and no
//   grid-wide synchronisation per round.
#include <algorithm>

#include "internal.hpp"

namespace flood {

static constexpr int kDenseBlock = 256;
static constexpr int kPT = 1024;          // persistent workgroup
static constexpr int kMaxChunks = 6144;   // chunk keys held in LDS per cloud (20 B each)

struct FpsState {
    int32_t cur;    // local index of the newest landmark
    float r2;       // current max of the running minima (covering radius squared)
    float lx, ly, lz;
    uint32_t done;  // blocks finished in a dense round
    int32_t shift;  // log2 of the chunk size
    int32_t nchunks;
    int64_t chunk_base;  // first chunk of this cloud in the global chunk arrays
};

struct FpsWork {
    GridWork grid;
    float *mind;      // [sum N] running minima, cell-sorted order
    uint64_t *ckey;   // [sum chunks]
    uint32_t *cpos;   // [sum chunks] position (within the cloud) of the chunk's argmax
    FpsState *state;  // [B]
    int64_t *l_off;   // [B+1]
};

static float fps_alpha() { return 1.0f; }

static int chunk_shift_host(int64_t n) {
    int s = 10;
    while (((n + (1ll << s) - 1) >> s) > kMaxChunks) ++s;
    return s;
}

static int64_t total_chunks_host(int32_t B, const int64_t *x_off) {
    int64_t c = 0;
    for (int32_t b = 0; b < B; ++b) {
        int64_t n = x_off[b + 1] - x_off[b];
        int s = chunk_shift_host(n);
        c += (n + (1ll << s) - 1) >> s;
    }
    return c;
}

size_t fps_workspace(int32_t B, const int64_t *x_off, const int32_t *n_lm) {
    (void)n_lm;
    int64_t tc = 0;
    size_t bytes = grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    const int64_t nc = total_chunks_host(B, x_off);
    bytes += sizeof(float) * np + 256;
    bytes += sizeof(uint64_t) * (nc + 1) + 256;
    bytes += sizeof(uint32_t) * (nc + 1) + 256;
    bytes += sizeof(FpsState) * B + 256;
    bytes += sizeof(int64_t) * (B + 1) + 256;
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

// max by key; the position travels with it
__device__ __forceinline__ void kp_max(uint64_t &k, uint32_t &p, uint64_t ok, uint32_t op) {
    if (ok > k) {
        k = ok;
        p = op;
    }
}

__device__ __forceinline__ void wave_kp_max(uint64_t &k, uint32_t &p) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t ok = __shfl_xor(k, o, 64);
        const uint32_t op = __shfl_xor(p, o, 64);
        kp_max(k, p, ok, op);
    }
}

// correctly rounded float sqrt: the double root is within one double ulp
// and the root of a float never lies that close to a float midpoint
__device__ __forceinline__ float sqrt_rn(float x) { return (float)sqrt((double)x); }

__global__ void k_fps_init(int32_t B, const int32_t *n_lm, const int64_t *start, const float *X, const int64_t *x_off,
                           FpsState *st, int64_t *l_off, int32_t *idx) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t o = 0, cb = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = x_off[b + 1] - x_off[b];
        int s = 10;
        while (((n + (1ll << s) - 1) >> s) > kMaxChunks) ++s;
        l_off[b] = o;
        FpsState S;
        S.cur = start ? (int32_t)start[b] : 0;
        const int64_t row = x_off[b] + S.cur;
        S.lx = X[3 * row];
        S.ly = X[3 * row + 1];
        S.lz = X[3 * row + 2];
        S.r2 = INFINITY;
        S.done = 0;
        S.shift = s;
        S.nchunks = (int32_t)((n + (1ll << s) - 1) >> s);
        S.chunk_base = cb;
        st[b] = S;
        idx[o] = S.cur;
        o += n_lm[b];
        cb += S.nchunks;
    }
    l_off[B] = o;
}

// ---------------------------------------------------------------------------
// dense round: gridDim = (max chunks per cloud, B); block = one chunk

__global__ __launch_bounds__(kDenseBlock) void k_fps_dense(
    int32_t t, const GridParam *__restrict__ gp, const float4 *__restrict__ xs, float *__restrict__ mind,
    uint64_t *__restrict__ ckey, uint32_t *__restrict__ cpos, FpsState *__restrict__ st,
    const int32_t *__restrict__ n_lm, const int64_t *__restrict__ l_off, int32_t *__restrict__ idx_out,
    float *__restrict__ radius) {
    const int b = blockIdx.y;
    if (t >= n_lm[b]) return;
    const FpsState S = st[b];
    const int c = blockIdx.x;
    if (c >= S.nchunks) return;
    const GridParam g = gp[b];
    const int64_t n = g.npts;
    const int64_t p0 = (int64_t)c << S.shift;
    const int64_t p1 = min(n, p0 + (1ll << S.shift));
    const uint32_t base_idx = (uint32_t)g.pt_base;
    uint64_t k = 0;
    uint32_t kp = 0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const float4 q = xs[g.pt_base + p];
        const float d2 = fps_d2(q.x, q.y, q.z, S.lx, S.ly, S.lz);
        float m = mind[g.pt_base + p];
        if (d2 < m) {
            m = d2;
            mind[g.pt_base + p] = m;
        }
        kp_max(k, kp, fps_key(m, (uint32_t)__float_as_int(q.w) - base_idx), (uint32_t)p);
    }
    wave_kp_max(k, kp);
    __shared__ uint64_t s_k[kDenseBlock / 64];
    __shared__ uint32_t s_p[kDenseBlock / 64];
    __shared__ uint32_t s_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        s_k[wid] = k;
        s_p[wid] = kp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kDenseBlock / 64; ++w) kp_max(k, kp, s_k[w], s_p[w]);
        ckey[S.chunk_base + c] = k;
        cpos[S.chunk_base + c] = kp;
        __threadfence();
        s_last = (atomicAdd(&st[b].done, 1u) == (uint32_t)S.nchunks - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // last block of the cloud: argmax over all chunk keys
    k = 0;
    kp = 0;
    for (int i = threadIdx.x; i < S.nchunks; i += blockDim.x) {
        const uint64_t v = __hip_atomic_load(&ckey[S.chunk_base + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t vp = __hip_atomic_load(&cpos[S.chunk_base + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        kp_max(k, kp, v, vp);
    }
    wave_kp_max(k, kp);
    __syncthreads();
    if (lane == 0) {
        s_k[wid] = k;
        s_p[wid] = kp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kDenseBlock / 64; ++w) kp_max(k, kp, s_k[w], s_p[w]);
        const float best = __uint_as_float((uint32_t)(k >> 32));
        const int32_t nxt = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
        const int64_t o = l_off[b];
        if (radius) radius[o + t] = sqrt_rn(best);
        if (t + 1 < n_lm[b]) idx_out[o + t + 1] = nxt;
        const float4 q = xs[g.pt_base + kp];
        st[b].cur = nxt;
        st[b].r2 = best;
        st[b].lx = q.x;
        st[b].ly = q.y;
        st[b].lz = q.z;
        st[b].done = 0;
    }
}

// ---------------------------------------------------------------------------
// persistent rounds: one workgroup per cloud, chunk keys in LDS

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

__global__ __launch_bounds__(kPT) void k_fps_persist(
    int32_t t0, const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs, const float4 *__restrict__ xs,
    float *__restrict__ mind, const uint64_t *__restrict__ ckey_g, const uint32_t *__restrict__ cpos_g,
    const FpsState *__restrict__ st, const int32_t *__restrict__ n_lm, const int64_t *__restrict__ l_off,
    int32_t *__restrict__ idx_out, float *__restrict__ radius) {
    extern __shared__ uint64_t s_dyn[];
    const int b = blockIdx.x;
    const int nl = n_lm[b];
    if (t0 >= nl) return;
    const FpsState S0 = st[b];
    const GridParam g = gp[b];
    const int nch = S0.nchunks;
    uint64_t *s_ckey = s_dyn;                                  // [nch]
    uint32_t *s_cpos = (uint32_t *)(s_ckey + nch);             // [nch]
    uint32_t *s_flag = s_cpos + nch;                           // [nch] (round stamp)
    uint32_t *s_list = s_flag + nch;                           // [nch] flagged chunks
    __shared__ uint32_t s_pa[kPT], s_off[kPT + 1], s_w[kPT / 64 + 1];
    __shared__ uint64_t s_rk[kPT / 64];
    __shared__ uint32_t s_rp[kPT / 64];
    __shared__ uint32_t s_nlist;
    __shared__ float s_l[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < nch; i += kPT) {
        s_ckey[i] = ckey_g[S0.chunk_base + i];
        s_cpos[i] = cpos_g[S0.chunk_base + i];
        s_flag[i] = 0xffffffffu;
    }
    if (tid == 0) {
        s_l[0] = S0.lx;
        s_l[1] = S0.ly;
        s_l[2] = S0.lz;
        s_l[3] = S0.r2;
        s_nlist = 0;
    }
    __syncthreads();
    const uint32_t base_idx = (uint32_t)g.pt_base;
    const int shift = S0.shift;
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
            float tl = fminf(fmaxf((l[a] - R - og[a]) * g.inv_h, -4.f), (float)n[a] + 4.f);
            float th = fminf(fmaxf((l[a] + R - og[a]) * g.inv_h, -4.f), (float)n[a] + 4.f);
            lo[a] = clampi((int)floorf(tl) - 1, 0, n[a] - 1);
            hi[a] = clampi((int)floorf(th) + 1, 0, n[a] - 1);
        }
        const int nyb = hi[1] - lo[1] + 1;
        const int nrows = nyb * (hi[2] - lo[2] + 1);
        for (int c0 = 0; c0 < nrows; c0 += kPT) {
            const int nr = min(kPT, nrows - c0);
            uint32_t cnt = 0;
            if (tid < nr) {
                const int r = c0 + tid;
                const int z = lo[2] + r / nyb, y = lo[1] + r % nyb;
                const int64_t rowcell = g.cell_base + ((int64_t)z * g.ny + y) * g.nx;
                const uint32_t pa = cs[rowcell + lo[0]];
                cnt = cs[rowcell + hi[0] + 1] - pa;
                s_pa[tid] = pa;
            }
            uint32_t total;
            const uint32_t off = block_scan_u32(cnt, &total, s_w);
            s_off[tid] = off;
            if (tid == kPT - 1) s_off[kPT] = total;
            __syncthreads();
#pragma unroll 4
            for (uint32_t k = tid; k < total; k += kPT) {
                int lo_r = 0, hi_r = nr;  // s_off[lo_r] <= k < s_off[hi_r]
                while (hi_r - lo_r > 1) {
                    const int mid = (lo_r + hi_r) >> 1;
                    if (s_off[mid] <= k) lo_r = mid;
                    else hi_r = mid;
                }
                const uint32_t p = s_pa[lo_r] + (k - s_off[lo_r]);  // global position
                const float4 q = xs[p];
                const float d2 = fps_d2(q.x, q.y, q.z, lx, ly, lz);
                const float m = mind[p];
                if (d2 < m) {
                    mind[p] = d2;
                    const uint32_t lp = p - base_idx;
                    const uint32_t c = lp >> shift;
                    if (s_cpos[c] == lp && atomicExch(&s_flag[c], (uint32_t)t) != (uint32_t)t) {
                        const uint32_t slot = atomicAdd(&s_nlist, 1u);
                        s_list[slot] = c;
                    }
                }
            }
            __syncthreads();
        }
        // recompute the flagged chunks (one wave per chunk)
        __threadfence_block();
        __syncthreads();
        const uint32_t nlist = s_nlist;
        for (uint32_t i = wid; i < nlist; i += kPT / 64) {
            const uint32_t c = s_list[i];
            const int64_t p0 = (int64_t)c << shift;
            const int64_t p1 = min((int64_t)g.npts, p0 + (1ll << shift));
            uint64_t k = 0;
            uint32_t kp = 0;
            for (int64_t p = p0 + lane; p < p1; p += 64) {
                const float m = mind[g.pt_base + p];
                const uint32_t li = (uint32_t)__float_as_int(xs[g.pt_base + p].w) - base_idx;
                kp_max(k, kp, fps_key(m, li), (uint32_t)p);
            }
            wave_kp_max(k, kp);
            if (lane == 0) {
                s_ckey[c] = k;
                s_cpos[c] = kp;
            }
        }
        __syncthreads();
        // argmax over the chunk keys
        uint64_t k = 0;
        uint32_t kp = 0;
        for (int i = tid; i < nch; i += kPT) kp_max(k, kp, s_ckey[i], s_cpos[i]);
        wave_kp_max(k, kp);
        if (lane == 0) {
            s_rk[wid] = k;
            s_rp[wid] = kp;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kPT / 64; ++w) kp_max(k, kp, s_rk[w], s_rp[w]);
            const float best = __uint_as_float((uint32_t)(k >> 32));
            const int32_t nxt = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
            if (radius) radius[o + t] = sqrt_rn(best);
            if (t + 1 < nl) idx_out[o + t + 1] = nxt;
            const float4 q = xs[g.pt_base + kp];
            s_l[0] = q.x;
            s_l[1] = q.y;
            s_l[2] = q.z;
            s_l[3] = best;
            s_nlist = 0;
        }
        __syncthreads();
    }
}

hipError_t fps_run(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                   const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                   float *radius, void *ws, size_t ws_bytes, hipStream_t s) {
    int64_t tc = 0;
    grid_workspace(B, x_off, fps_alpha(), &tc);
    const int64_t np = x_off[B];
    const int64_t nc = total_chunks_host(B, x_off);
    Carve c(ws, ws_bytes);
    FpsWork w;
    grid_carve(c, B, np, tc, w.grid);
    w.mind = c.take<float>(np);
    w.ckey = c.take<uint64_t>(nc + 1);
    w.cpos = c.take<uint32_t>(nc + 1);
    w.state = c.take<FpsState>(B);
    w.l_off = c.take<int64_t>(B + 1);
    if (!c.ok()) return hipErrorOutOfMemory;
    hipError_t e = grid_build(X, B, x_off, x_off_d, fps_alpha(), w.grid, s);
    if (e != hipSuccess) return e;
    e = fill_f32(w.mind, INFINITY, np, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fps_init, dim3(1), dim3(1), 0, s, B, n_lm_d, start_d, X, x_off_d, w.state, w.l_off, idx);
    int64_t nmax = 0;
    int32_t rounds = 0, max_chunks = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = x_off[b + 1] - x_off[b];
        nmax = n > nmax ? n : nmax;
        rounds = n_lm[b] > rounds ? n_lm[b] : rounds;
        const int sh = chunk_shift_host(n);
        max_chunks = std::max<int32_t>(max_chunks, (int32_t)((n + (1ll << sh) - 1) >> sh));
    }
    // dense rounds while a round touches most of a large cloud, then one
    // persistent workgroup per cloud
    const int32_t t0 = std::min<int32_t>(rounds, nmax > 2000000 ? 24 : 1);
    for (int32_t t = 0; t < t0; ++t)
        hipLaunchKernelGGL(k_fps_dense, dim3(max_chunks, B), dim3(kDenseBlock), 0, s, t, w.grid.gp, w.grid.xs, w.mind,
                           w.ckey, w.cpos, w.state, n_lm_d, w.l_off, idx, radius);
    if (t0 < rounds) {
        const size_t lds = (size_t)max_chunks * (sizeof(uint64_t) + 3 * sizeof(uint32_t));
        hipLaunchKernelGGL(k_fps_persist, dim3(B), dim3(kPT), lds, s, t0, w.grid.gp, w.grid.cell_start, w.grid.xs,
                           w.mind, w.ckey, w.cpos, w.state, n_lm_d, w.l_off, idx, radius);
    }
    return hipGetLastError();
}

}  // namespace flood
