// The flooding step: for every simplex sigma of Del(L), the sampled flood
// value f(sigma) = max_{tau face of sigma} max_{p in P_tau} min_{x in X} ||p-x||
// (Def. 1, Sec. 4.1; P_tau the barycentric grid of Lemma 6, k segments per
// edge).  Dimensions run bottom-up.  A simplex only evaluates its INTERIOR
// samples (all a_i >= 1): the samples on its boundary belong to its facets,
// whose values arrive as the seed M = max over facets f(tau) -- the closure
// of Sec. 4.1, and exactly the max over the full grid because P_tau is a
// subset of P_sigma.
//
// Search, phase A (one wavefront per tile of 64*T samples, or of 16 or 32
// samples held by 4 or 2 lanes each, consecutive in Morton order, so a tile
// is spatially compact; the sample sort computes every sample's point and
// bound once):
//  * each sample starts from the bound d(p,X)^2 <= min_i |p - v_i|^2, valid
//    when the landmarks are points of X (proof of Lemma 7);
//  * the wave scans grid cells in growing boxes around its samples, one
//    x-run of cells (contiguous points) per lane; a run is kept only if
//    some live sample's distance to the run's box is below its bound; the
//    kept runs' points are loaded 64 at a time with one coalesced load,
//    staged in LDS and read back at one address by every lane, which
//    updates its minimum with direct-difference FP32;
//  * a sample retires as soon as its bound drops below the simplex's
//    running max M (it cannot raise f), and completes when its bound is
//    below the distance to the unscanned region (its minimum is exact);
//  * completed samples above the seed publish (value, rank) with a 64-bit
//    atomic max per simplex, which other tiles read to raise M.
// Phase B takes the samples a tile left open, one wavefront each, in rings
// of grid rows around the sample; it keeps the nearest point's row, which
// becomes x* when the sample wins.  The remaining winners get x* from a
// search with the known value as radius.
// Every skip is conservative, so the result equals the unpruned max-min.
#include "sample.hpp"

namespace flood {

static constexpr int kWaveBlock = 256;
static constexpr int kTileLanesDefault[4] = {64, 64, 64, 64};  // samples per tile of the tile search, by dimension
static constexpr uint32_t kFineMin = 8;  // shortest cell run the tile search tests against every sample
static constexpr int kU = 2;  // points per lane per step in the per-sample search
static constexpr int kStage = 128;  // points staged in LDS per pass of the tile search

// an open sample handed from phase A to phase B: its position and distance
// bound, its id (simplex * interior samples + rank) and cloud
struct __align__(16) OpenSample {
    float4 p;  // x, y, z, squared-distance bound
    uint32_t gid, cloud;
    // after the per-sample search: the nearest point's row and the value
    // (float bits) when the search ran to the end, kNoRow otherwise
    uint32_t xrow, val;
};
static constexpr uint32_t kNoRow = 0xffffffffu;

// ---------------------------------------------------------------------------
// per-dimension helpers

// tile offsets per cloud: tiles_b = ceil(n_b * n_int / (64 T)) (one block,
// a thread per cloud in rounds)
// the cloud of every tile (batched calls): a binary search over the tile
// offsets once per tile here, instead of a chain of dependent loads at the
// start of every tile wavefront
__global__ void k_tile_cloud(const int64_t *__restrict__ tile_off, int32_t B, int64_t n_tiles,
                             uint32_t *__restrict__ tcloud) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    int lo_b = 0, hi_b = B;
    while (hi_b - lo_b > 1) {
        const int mid = (lo_b + hi_b) >> 1;
        if (tile_off[mid] <= t) lo_b = mid;
        else hi_b = mid;
    }
    tcloud[t] = (uint32_t)lo_b;
}

__global__ __launch_bounds__(1024) void k_tile_off(const int64_t *s_off, int32_t B, int64_t n_int,
                                                    int64_t tile_samples, int64_t *tile_off) {
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < B; b0 += (int32_t)blockDim.x) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const int64_t S = b < B ? (s_off[b + 1] - s_off[b]) * n_int : 0;
        int64_t total;
        const int64_t off = block_exclusive_i64((S + tile_samples - 1) / tile_samples, total);
        if (b < B) tile_off[b] = carry + off;
        carry += total;
    }
    if (threadIdx.x == 0) tile_off[B] = carry;
}

// seed = max over facets (facet i omits vertex i); 0 for vertices
__global__ void k_seed(int d, int64_t n, const int32_t *__restrict__ simp1, const int32_t *__restrict__ tri_edges,
                       const int32_t *__restrict__ tet_tris, const float *__restrict__ fprev, float *__restrict__ seed) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float m = 0.f;
    if (d == 1) {
        m = fmaxf(fprev[simp1[2 * j]], fprev[simp1[2 * j + 1]]);
    } else if (d == 2) {
        m = fmaxf(fmaxf(fprev[tri_edges[3 * j]], fprev[tri_edges[3 * j + 1]]), fprev[tri_edges[3 * j + 2]]);
    } else if (d == 3) {
        m = fmaxf(fmaxf(fprev[tet_tris[4 * j]], fprev[tet_tris[4 * j + 1]]),
                  fmaxf(fprev[tet_tris[4 * j + 2]], fprev[tet_tris[4 * j + 3]]));
    }
    seed[j] = m;
}

__device__ __forceinline__ float key_value(uint64_t kv) { return __uint_as_float((uint32_t)(kv >> 32)); }

// ---------------------------------------------------------------------------
// sample order: a counting sort of each dimension's interior samples by the
// Morton code of their position on a per-cloud 2^m cube (m chosen for about
// four samples per bucket), so that 64 consecutive samples form a compact
// tile whatever simplices they come from.

__global__ __launch_bounds__(1024) void k_bucket_base(const int64_t *s_off, int32_t B, int64_t n_int, int32_t *mbits,
                                                       uint32_t *bbase) {
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < B; b0 += (int32_t)blockDim.x) {
        const int32_t b = b0 + (int32_t)threadIdx.x;
        const int m = b < B ? morton_bits((s_off[b + 1] - s_off[b]) * n_int) : 0;
        int64_t total;
        const int64_t off = block_exclusive_i64(b < B ? (int64_t)1 << (3 * m) : 0, total);
        if (b < B) {
            mbits[b] = m;
            bbase[b] = (uint32_t)(carry + off);
        }
        carry += total;
    }
    if (threadIdx.x == 0) bbase[B] = (uint32_t)carry;
}

// the cloud of every simplex of a dimension (batched calls), once per
// simplex instead of once per sample
__global__ void k_simplex_cloud(const int64_t *__restrict__ s_off, int32_t B, int64_t n, uint32_t *__restrict__ scloud) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int lo_b = 0, hi_b = B;
    while (hi_b - lo_b > 1) {
        const int mid = (lo_b + hi_b) >> 1;
        if (s_off[mid] <= j) lo_b = mid;
        else hi_b = mid;
    }
    scloud[j] = (uint32_t)lo_b;
}

__global__ void k_sample_keys(int d, SampleRule rule, int n_int, int32_t B, int64_t S, const float *__restrict__ L,
                              const int32_t *__restrict__ simp, const int64_t *__restrict__ s_off,
                              const uint32_t *__restrict__ scloud,
                              const GridParam *__restrict__ gp, const int32_t *__restrict__ mbits,
                              const uint32_t *__restrict__ bbase, const float *__restrict__ X,
                              const int32_t *__restrict__ l_xidx, const int64_t *__restrict__ x_off,
                              int32_t landmarks_in_x, uint32_t *__restrict__ skey, uint32_t *__restrict__ srank,
                              uint32_t *__restrict__ counts, float4 *__restrict__ spos) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= S) return;
    const int64_t j = gid / n_int;
    const int q = (int)(gid % n_int);
    const int lo_b = B == 1 ? 0 : (int)scloud[j];
    const GridParam g = gp[lo_b];
    float w[4];
    own_weights(rule, d, q, j - s_off[lo_b], w);
    int32_t v[4];
    simplex_vertices(simp, d, j, v);
    float sx, sy, sz;
    weighted_point(L, v, w, d, sx, sy, sz);
    float u = INFINITY;
    if (landmarks_in_x) {
        // the squared distance to the vertices' own points of X (read from
        // X, so it holds whatever the landmark array holds; a row outside
        // the cloud gives no bound): an upper bound of the sample's value
        const int64_t x_lo = x_off[lo_b], x_hi = x_off[lo_b + 1];
        for (int i = 0; i <= d; ++i) {
            const int64_t xi = l_xidx[v[i]];
            if (xi >= x_lo && xi < x_hi) u = fminf(u, dist2(sx, sy, sz, X[3 * xi], X[3 * xi + 1], X[3 * xi + 2]));
        }
    }
    spos[gid] = make_float4(sx, sy, sz, u);
    const int m = mbits[lo_b];
    const float ext = (float)max(max(g.nx, g.ny), g.nz) * g.h;
    const float sc = (float)(1 << m) / ext;
    const int top = (1 << m) - 1;
    const int qx = min(max((int)((sx - g.ox) * sc), 0), top);
    const int qy = min(max((int)((sy - g.oy) * sc), 0), top);
    const int qz = min(max((int)((sz - g.oz) * sc), 0), top);
    const uint32_t key = bbase[lo_b] + (spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2));
    skey[gid] = key;
    // the sample's place in its bucket: one atomic per distinct key of the
    // wavefront (neighbouring samples share buckets)
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(true);
    while (todo) {
        const int ldr = __ffsll((unsigned long long)todo) - 1;
        const uint32_t kl = __builtin_amdgcn_readlane(key, ldr);
        const uint64_t same = __ballot(key == kl) & todo;
        uint32_t base = 0;
        if (lane == ldr) base = atomicAdd(&counts[kl], (uint32_t)__popcll(same));
        base = __shfl(base, ldr, 64);
        if ((same >> lane) & 1ull) srank[gid] = base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
}

__global__ void k_sample_scatter(int64_t S, const uint32_t *__restrict__ skey, const uint32_t *__restrict__ srank,
                                 const uint32_t *__restrict__ bstart, uint32_t *__restrict__ order) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= S) return;
    order[bstart[skey[gid]] + srank[gid]] = (uint32_t)gid;
}

// ---------------------------------------------------------------------------
// phase A: cooperative tile scan (compact tiles, bounded radius)

struct TileArgs {
    int32_t d, k, n_int, landmarks_in_x;
    int32_t B, radius_budget;  // shells scanned beyond the samples' own cells
    int32_t max_extent;        // tiles whose samples span more cells go straight to phase B
    int32_t sampling;
    int64_t n_tiles;
    uint64_t seed;
    int32_t lanes;             // samples per tile (64, or with T = 1: 32 or 16, each held by 64/lanes lanes)
    int32_t pad;
};

__device__ __forceinline__ float box_lb2(float sx, float sy, float sz, float bx0, float bx1, float by0, float by1,
                                         float bz0, float bz1) {
    const float ex = fmaxf(fmaxf(bx0 - sx, sx - bx1), 0.f);
    const float ey = fmaxf(fmaxf(by0 - sy, sy - by1), 0.f);
    const float ez = fmaxf(fmaxf(bz0 - sz, sz - bz1), 0.f);
    return ex * ex + ey * ey + ez * ez;
}

// `always`: vertices publish their value whatever the seed; `own_ties`:
// random sets, whose own samples win a tie with the facets (the grid's
// facets hold those samples themselves)
__device__ __forceinline__ void publish(uint64_t *key, const float *seed, int32_t j, int32_t q, float best,
                                        bool always, bool own_ties) {
    const float v = sqrt_rn(best);
    if (always || v > seed[j] || (own_ties && v == seed[j])) {
        const uint64_t nk = ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)(0xffffffffu - (uint32_t)q);
        atomicMax((unsigned long long *)&key[j], (unsigned long long)nk);
    }
}

template <int T>
__global__ __launch_bounds__(kWaveBlock) __attribute__((amdgpu_waves_per_eu(T == 1 ? 8 : 1, 8))) void k_flood_tiles(
    TileArgs a, const float4 *__restrict__ spos, const int64_t *__restrict__ s_off,
    const int64_t *__restrict__ tile_off, const uint32_t *__restrict__ tcloud, const float *__restrict__ seed,
    uint64_t *__restrict__ key,
    const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs, const float4 *__restrict__ xs,
    const uint32_t *__restrict__ order, OpenSample *__restrict__ hard, uint32_t *__restrict__ hard_count,
    unsigned long long *__restrict__ evals, unsigned long long *__restrict__ stats) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    // staged points, coordinates apart: one 16-byte read gives a coordinate of four points
    __shared__ __align__(16) float s_px[kWaveBlock / 64][3][kStage];
    __shared__ uint32_t s_p0[kWaveBlock / 64][64], s_end[kWaveBlock / 64][64];
    float *sw_x = s_px[threadIdx.x >> 6][0], *sw_y = s_px[threadIdx.x >> 6][1], *sw_z = s_px[threadIdx.x >> 6][2];
    uint32_t *sw_p0 = s_p0[threadIdx.x >> 6], *sw_end = s_end[threadIdx.x >> 6];
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // tile state in scalar registers
    const int64_t wave = xcd_remap(blockIdx.x, gridDim.x) * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= a.n_tiles) return;
    const int b = a.B == 1 ? 0 : (int)__builtin_amdgcn_readfirstlane(tcloud[wave]);
    const GridParam g = gp[b];
    const int64_t sbase = s_off[b];
    const int64_t S = (s_off[b + 1] - sbase) * (int64_t)a.n_int;
    // a tile of a.lanes samples (T = 1; 64 T otherwise); with fewer than 64,
    // lane l holds sample l mod a.lanes, a copy that scans its share of every
    // staged pass from the start (see grp below)
    const int tl = T == 1 ? a.lanes : 64;
    const int64_t ls0 = (wave - tile_off[b]) * (int64_t)tl * T;
    const int d = a.d;

    float sx[T], sy[T], sz[T], best[T], M[T];
    int32_t sj[T], sq[T];
    bool live[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t ls = ls0 + (int64_t)t * 64 + (lane & (tl - 1));
        const bool valid = ls < S;
        sx[t] = sy[t] = sz[t] = 0.f;
        best[t] = 0.f;
        M[t] = 0.f;
        sj[t] = 0;
        sq[t] = 0;
        if (valid) {
            // the sample's point and its bound, from the sample sort (in
            // global sample order: simplex j's samples from j * n_int on)
            const uint32_t gid = order[sbase * a.n_int + ls];
            const int64_t j = gid / (uint32_t)a.n_int;
            const int q = (int)(gid % (uint32_t)a.n_int);
            sj[t] = (int32_t)j;
            sq[t] = q;
            const float4 sp = spos[gid];
            sx[t] = sp.x;
            sy[t] = sp.y;
            sz[t] = sp.z;
            best[t] = sp.w;
            M[t] = seed[j];
        }
        live[t] = valid && !(sqrt_rn(best[t]) < M[t]);
        if (live[t] && best[t] == 0.f) {
            // a sample on a point of X: its value 0 is exact (a vertex sample)
            if (lane < tl) publish(key, seed, sj[t], sq[t], 0.f, d == 0, a.sampling == FLOOD_SAMPLING_RANDOM);
            live[t] = false;
        }
    }
    const float h = g.h, eps = g.eps;
    // initial box: the cells of the live samples
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (live[t]) {
            const int cx = cell_of(sx[t], g.ox, g.inv_h, g.nx);
            const int cy = cell_of(sy[t], g.oy, g.inv_h, g.ny);
            const int cz = cell_of(sz[t], g.oz, g.inv_h, g.nz);
            lo[0] = min(lo[0], cx); hi[0] = max(hi[0], cx);
            lo[1] = min(lo[1], cy); hi[1] = max(hi[1], cy);
            lo[2] = min(lo[2], cz); hi[2] = max(hi[2], cz);
        }
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo[ax] = min(lo[ax], __shfl_xor(lo[ax], o, 64));
            hi[ax] = max(hi[ax], __shfl_xor(hi[ax], o, 64));
        }
        lo[ax] = __builtin_amdgcn_readfirstlane(lo[ax]);
        hi[ax] = __builtin_amdgcn_readfirstlane(hi[ax]);
    }
    unsigned long long nev = 0, nslot = 0;  // evaluations of live samples; of all the tile's sample slots
    // lanes [0, grp) hold the tile's samples; with grp < 64 (one sample per
    // lane only) lane l holds a copy of lane l mod grp's sample and scans its
    // share of every staged pass, and the copies' minima are combined after
    // each shell
    int grp = tl;
    const bool any_live = hi[0] >= 0;
    const bool compact = any_live && hi[0] - lo[0] < a.max_extent && hi[1] - lo[1] < a.max_extent &&
                         hi[2] - lo[2] < a.max_extent && a.radius_budget >= 0;
    if (compact) {
        int olo[3] = {lo[0], lo[1], lo[2]}, ohi[3] = {lo[0] - 1, lo[1] - 1, lo[2] - 1};  // empty old box
        // live-sample bounding box (a coarse cull for the rows), recomputed
        // only when the set of live lanes changed: a stale box is larger,
        // which culls less but never wrongly
        float lx0 = 0.f, lx1 = 0.f, ly0 = 0.f, ly1 = 0.f, lz0 = 0.f, lz1 = 0.f;
        uint64_t box_live = 0;
        for (int r = 0;; ++r) {
            float bmax = 0.f;
#pragma unroll
            for (int t = 0; t < T; ++t)
                if (live[t]) bmax = fmaxf(bmax, best[t]);
            const uint64_t now_live = __ballot(live[0]);
            if (T > 1 || r == 0 || now_live != box_live) {
                box_live = now_live;
                lx0 = INFINITY; lx1 = -INFINITY; ly0 = INFINITY; ly1 = -INFINITY; lz0 = INFINITY; lz1 = -INFINITY;
#pragma unroll
                for (int t = 0; t < T; ++t)
                    if (live[t]) {
                        lx0 = fminf(lx0, sx[t]); lx1 = fmaxf(lx1, sx[t]);
                        ly0 = fminf(ly0, sy[t]); ly1 = fmaxf(ly1, sy[t]);
                        lz0 = fminf(lz0, sz[t]); lz1 = fmaxf(lz1, sz[t]);
                    }
                lx0 = wave_min_f32_dpp(lx0); lx1 = wave_max_f32_dpp(lx1);
                ly0 = wave_min_f32_dpp(ly0); ly1 = wave_max_f32_dpp(ly1);
                lz0 = wave_min_f32_dpp(lz0); lz1 = wave_max_f32_dpp(lz1);
            }
            // the largest bound falls every shell
            bmax = wave_max_f32_dpp(bmax);
            // rows of box [lo,hi] minus box [olo,ohi], enumerated 64 at a time
            const int nyb = hi[1] - lo[1] + 1;
            const int nrows = nyb * (hi[2] - lo[2] + 1);
            for (int base = 0; base < nrows; base += 64) {
                const int i = base + lane;
                const int y = lo[1] + i % nyb, z = lo[2] + i / nyb;
                const bool inner = r > 0 && z >= olo[2] && z <= ohi[2] && y >= olo[1] && y <= ohi[1];
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                    int x0, x1;
                    if (!inner) {
                        x0 = lo[0];
                        x1 = part ? lo[0] - 1 : hi[0];
                    } else if (part == 0) {
                        x0 = lo[0];
                        x1 = olo[0] - 1;
                    } else {
                        x0 = ohi[0] + 1;
                        x1 = hi[0];
                    }
                    bool ok = i < nrows && x0 <= x1;
                    uint32_t p0 = 0, p1 = 0;
                    if (ok) {
                        const int64_t c0 = g.cell_base + ((int64_t)z * g.ny + y) * g.nx + x0;
                        p0 = cs[c0];
                        p1 = cs[c0 + (x1 - x0) + 1];
                        ok = p1 > p0;
                    }
                    if (ok) {
                        // coarse: distance between the run's box and the live samples' box
                        const float gx = fmaxf(fmaxf((g.ox + (float)x0 * h - eps) - lx1, lx0 - (g.ox + (float)(x1 + 1) * h + eps)), 0.f);
                        const float gy = fmaxf(fmaxf((g.oy + (float)y * h - eps) - ly1, ly0 - (g.oy + (float)(y + 1) * h + eps)), 0.f);
                        const float gz = fmaxf(fmaxf((g.oz + (float)z * h - eps) - lz1, lz0 - (g.oz + (float)(z + 1) * h + eps)), 0.f);
                        ok = gx * gx + gy * gy + gz * gz < bmax;
                    }
                    // fine: keep a run only if some live sample's bound reaches its box
                    // (a run shorter than kFineMin points is kept: testing it costs more
                    // than scanning it)
                    uint64_t mask = __ballot(ok && p1 - p0 >= kFineMin), need_m = __ballot(ok && p1 - p0 < kFineMin);
                    if (T == 1 && grp < 64 && mask) {
                        // every group of grp lanes holds each of the tile's
                        // samples once, so the groups test 64 / grp runs at
                        // a time: group c takes run c of the round
                        const int nm = __popcll(mask);
                        const int lg = __builtin_ctz((unsigned)grp);
                        if ((mask >> lane) & 1ull) sw_p0[__popcll(mask & ((1ull << lane) - 1ull))] = (uint32_t)lane;
                        sw_end[lane] = 0u;
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        for (int r0 = 0; r0 < nm; r0 += 64 >> lg) {
                            const int idx = r0 + (lane >> lg);
                            const int src = idx < nm ? (int)sw_p0[idx] : 0;
                            const int rx0 = __shfl(x0, src, 64), rx1 = __shfl(x1, src, 64);
                            const int ry = __shfl(y, src, 64), rz = __shfl(z, src, 64);
                            bool need = false;
                            if (idx < nm && live[0]) {
                                const float bx0 = g.ox + (float)rx0 * h - eps, bx1 = g.ox + (float)(rx1 + 1) * h + eps;
                                const float by0 = g.oy + (float)ry * h - eps, by1 = g.oy + (float)(ry + 1) * h + eps;
                                const float bz0 = g.oz + (float)rz * h - eps, bz1 = g.oz + (float)(rz + 1) * h + eps;
                                need = box_lb2(sx[0], sy[0], sz[0], bx0, bx1, by0, by1, bz0, bz1) < best[0];
                            }
                            const uint64_t bm = __ballot(need);
                            const uint64_t gbits = (bm >> (lane & ~(grp - 1))) & ((1ull << grp) - 1ull);
                            if (idx < nm && (lane & (grp - 1)) == 0 && gbits) sw_end[src] = 1u;
                        }
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        need_m |= __ballot(sw_end[lane] != 0u);
                        __builtin_amdgcn_wave_barrier();
                        mask = 0;
                    }
                    while (mask) {
                        const int src = __ffsll((unsigned long long)mask) - 1;
                        mask &= mask - 1;
                        const int rx0 = __builtin_amdgcn_readlane(x0, src);
                        const int rx1 = __builtin_amdgcn_readlane(x1, src);
                        const int ry = __builtin_amdgcn_readlane(y, src);
                        const int rz = __builtin_amdgcn_readlane(z, src);
                        const float bx0 = g.ox + (float)rx0 * h - eps, bx1 = g.ox + (float)(rx1 + 1) * h + eps;
                        const float by0 = g.oy + (float)ry * h - eps, by1 = g.oy + (float)(ry + 1) * h + eps;
                        const float bz0 = g.oz + (float)rz * h - eps, bz1 = g.oz + (float)(rz + 1) * h + eps;
                        bool need = false;
#pragma unroll
                        for (int t = 0; t < T; ++t)
                            if (live[t]) need |= box_lb2(sx[t], sy[t], sz[t], bx0, bx1, by0, by1, bz0, bz1) < best[t];
                        if (__any(need)) need_m |= 1ull << src;
                    }
                    if (!need_m) continue;
                    int nlive = 0;
#pragma unroll
                    for (int t = 0; t < T; ++t) nlive += __popcll(__ballot(live[t] && lane < grp));
                    // the kept runs' points, flattened: 64 per coalesced load,
                    // staged in LDS and read back at one address by every lane
                    const uint32_t cnt = ((need_m >> lane) & 1ull) ? p1 - p0 : 0u;
                    const uint32_t incl = wave_incl_sum(cnt);
                    const uint32_t total = rd_lane(incl, 63);
                    sw_p0[lane] = p0;
                    sw_end[lane] = incl;
                    nev += (unsigned long long)total * (unsigned long long)nlive;
                    nslot += (unsigned long long)total * (unsigned long long)(T * grp);
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    // kStage points per pass (kStage / 64 per lane); the next
                    // pass's loads are issued before this pass is evaluated
                    auto fetch = [&](uint32_t b0, float4 (&c)[kStage / 64]) {
#pragma unroll
                        for (int u = 0; u < kStage / 64; ++u) {
                            const uint32_t k = b0 + (uint32_t)(u * 64 + lane);
                            c[u] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
                            if (k < total) {
                                // first run whose inclusive end exceeds k (ends are
                                // non-decreasing; k < total, the last end): six fixed steps
                                int rr = 0;
#pragma unroll
                                for (int st = 32; st > 0; st >>= 1) rr += sw_end[rr + st - 1] <= k ? st : 0;
                                c[u] = xs[sw_p0[rr] + (k - (rr ? sw_end[rr - 1] : 0u))];
                            }
                        }
                    };
                    float4 cn[kStage / 64];
                    fetch(0, cn);
                    for (uint32_t b0 = 0; b0 < total; b0 += kStage) {
                        float4 cc[kStage / 64];
#pragma unroll
                        for (int u = 0; u < kStage / 64; ++u) cc[u] = cn[u];
                        if (b0 + kStage < total) fetch(b0 + kStage, cn);
                        __builtin_amdgcn_wave_barrier();
#pragma unroll
                        for (int u = 0; u < kStage / 64; ++u) {
                            sw_x[u * 64 + lane] = cc[u].x;
                            sw_y[u * 64 + lane] = cc[u].y;
                            sw_z[u * 64 + lane] = cc[u].z;
                        }
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        const int n4 = (int)((min(total - b0, (uint32_t)kStage) + 3u) & ~3u);
                        auto eval4 = [&](int j) {
                            const float4 px = *(const float4 *)&sw_x[j], py = *(const float4 *)&sw_y[j],
                                         pz = *(const float4 *)&sw_z[j];
#pragma unroll
                            for (int t = 0; t < T; ++t) {
                                const float d0 = dist2(sx[t], sy[t], sz[t], px.x, py.x, pz.x);
                                const float d1 = dist2(sx[t], sy[t], sz[t], px.y, py.y, pz.y);
                                const float d2 = dist2(sx[t], sy[t], sz[t], px.z, py.z, pz.z);
                                const float d3 = dist2(sx[t], sy[t], sz[t], px.w, py.w, pz.w);
                                best[t] = fminf(fminf(best[t], d0), d1);  // two v_min3
                                best[t] = fminf(fminf(best[t], d2), d3);
                            }
                        };
                        if (grp == 64) {
                            for (int j = 0; j < n4; j += 4) eval4(j);
                        } else {
                            // copy c = lane / grp takes the groups of four c, c + 64/grp, ...
                            const int jstep = 256 / grp;
                            for (int j = 4 * (lane / grp); j < n4; j += jstep) eval4(j);
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
            if (T == 1 && grp < 64) {
                // the copies' minima: lanes l and l ^ o (o >= grp) hold the same sample
                for (int o = grp; o < 64; o <<= 1) best[0] = fminf(best[0], __shfl_xor(best[0], o, 64));
            }
            // completion and retirement
            const bool full = lo[0] == 0 && lo[1] == 0 && lo[2] == 0 && hi[0] == g.nx - 1 && hi[1] == g.ny - 1 &&
                              hi[2] == g.nz - 1;
            bool anylive = false;
#pragma unroll
            for (int t = 0; t < T; ++t) {
                if (!live[t]) continue;
                float ext = INFINITY;
                if (!full) {
                    if (lo[0] > 0) ext = fminf(ext, sx[t] - (g.ox + (float)lo[0] * h));
                    if (hi[0] < g.nx - 1) ext = fminf(ext, (g.ox + (float)(hi[0] + 1) * h) - sx[t]);
                    if (lo[1] > 0) ext = fminf(ext, sy[t] - (g.oy + (float)lo[1] * h));
                    if (hi[1] < g.ny - 1) ext = fminf(ext, (g.oy + (float)(hi[1] + 1) * h) - sy[t]);
                    if (lo[2] > 0) ext = fminf(ext, sz[t] - (g.oz + (float)lo[2] * h));
                    if (hi[2] < g.nz - 1) ext = fminf(ext, (g.oz + (float)(hi[2] + 1) * h) - sz[t]);
                    ext -= eps;
                }
                const bool complete = full || (ext > 0.f && best[t] <= ext * ext);
                if (complete) {
                    // exact minimum: publish (value, rank); x* is found later
                    // for the winning sample only
                    live[t] = false;
                    if (lane < grp) publish(key, seed, sj[t], sq[t], best[t], d == 0, a.sampling == FLOOD_SAMPLING_RANDOM);
                } else {
                    const uint64_t kv = __hip_atomic_load(&key[sj[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    M[t] = fmaxf(M[t], key_value(kv));
                    if (sqrt_rn(best[t]) < M[t]) live[t] = false;
                }
                anylive |= live[t];
            }
            if (T == 1 && grp < 64) {
                // the copies follow their sample's own lane (the running
                // values they loaded may differ)
                const int c = lane & (grp - 1);
                live[0] = __shfl((int)live[0], c, 64) != 0;
                M[0] = __shfl(M[0], c, 64);
                anylive = live[0];
            }
            if (!__any(anylive) || full || r >= a.radius_budget) break;
            if (T == 1) {
                // at most half the samples still open: gather them into the
                // lowest lanes and give each 64 / grp copies
                const uint64_t lm = __ballot(live[0] && lane < grp);
                const int n = __popcll(lm);
                int ng = 2;
                while (ng < n) ng <<= 1;
                if (ng < grp) {
                    if (live[0] && lane < grp) sw_p0[__popcll(lm & ((1ull << lane) - 1ull))] = (uint32_t)lane;
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    const int idx = lane & (ng - 1);
                    const int src = idx < n ? (int)sw_p0[idx] : 0;
                    __builtin_amdgcn_wave_barrier();
                    sx[0] = __shfl(sx[0], src, 64);
                    sy[0] = __shfl(sy[0], src, 64);
                    sz[0] = __shfl(sz[0], src, 64);
                    best[0] = __shfl(best[0], src, 64);
                    M[0] = __shfl(M[0], src, 64);
                    sj[0] = __shfl(sj[0], src, 64);
                    sq[0] = __shfl(sq[0], src, 64);
                    live[0] = idx < n;
                    grp = ng;
                }
            }
            for (int ax = 0; ax < 3; ++ax) {
                olo[ax] = lo[ax];
                ohi[ax] = hi[ax];
            }
            lo[0] = max(lo[0] - 1, 0); hi[0] = min(hi[0] + 1, g.nx - 1);
            lo[1] = max(lo[1] - 1, 0); hi[1] = min(hi[1] + 1, g.ny - 1);
            lo[2] = max(lo[2] - 1, 0); hi[2] = min(hi[2] + 1, g.nz - 1);
        }
    }
    // open samples go to phase B with their bound
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const bool push = live[t] && lane < grp;
        const uint64_t m = __ballot(push);
        if (!m) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(hard_count, (uint32_t)__popcll(m));
        base = __shfl(base, 0, 64);
        if (push) {
            const uint32_t slot = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            OpenSample o;
            o.p = make_float4(sx[t], sy[t], sz[t], best[t]);
            o.gid = (uint32_t)(sj[t] * (int64_t)a.n_int + sq[t]);
            o.cloud = (uint32_t)b;
            o.xrow = kNoRow;
            o.val = 0u;
            hard[slot] = o;
        }
    }
    if (evals && lane == 0 && nev) atomicAdd(evals, nev);
    if (stats && lane == 0 && nev) atomicAdd(&stats[4 * d + 2], nev);
    if (stats && lane == 0 && nslot) atomicAdd(&stats[16 + 4 * d], nslot);
}

// ---------------------------------------------------------------------------
// phase B: one wavefront per open sample.  The lanes take the rows (y,z) of
// the grid in Chebyshev rings around the sample's cell, 64 rows per round
// trip; each row contributes the x-range that can beat the current bound,
// the rows' points are flattened over the lanes and every lane keeps its
// minimum d^2 (the winner search, which reuses the walk, keeps the
// lexicographic minimum (d^2, point row)); a wave reduction after every step
// shares the bound.  (Wider steps scan more points: the rows of one step
// share the bound from its start.)  Ring r cannot hold a point closer than
// (r-1) h, which ends the search.

struct DeepArgs {
    int32_t d, k, n_int, B;
    uint32_t grab;  // queue entries per atomic; 0: kGrab above 2^19 open samples, else kGrabSmall
    int32_t sampling;
};

__device__ __forceinline__ void ring_pos(int i, int &r, int &dy, int &dz) {
    // i-th row in ring order: ring r holds 8r rows (1 for r = 0) and starts
    // at index (2r-1)^2; its four sides of 2r rows each, without branches
    // (sqrt of i + 1/2 lands within one ring of the answer; one step fixes it)
    int rr = (int)((sqrtf((float)i + 0.5f) + 1.0f) * 0.5f);
    rr -= (2 * rr - 1) * (2 * rr - 1) > i ? 1 : 0;
    rr += (2 * rr + 1) * (2 * rr + 1) <= i ? 1 : 0;
    const int e = 2 * rr;
    const int p = i - (e - 1) * (e - 1);
    const int side = (p >= e ? 1 : 0) + (p >= 2 * e ? 1 : 0) + (p >= 3 * e ? 1 : 0);
    const int off = p - side * e;
    const int lo = off - rr, hi = rr - off;
    dy = side == 0 ? lo : (side == 1 ? rr : (side == 2 ? hi : -rr));
    dz = side == 0 ? -rr : (side == 1 ? lo : (side == 2 ? rr : hi));
    if (i == 0) {
        rr = 0;
        dy = 0;
        dz = 0;
    }
    r = rr;
}

__device__ __forceinline__ void lex_min(float &bd, int32_t &bi, float od, int32_t oi) {
    if (od < bd || (od == bd && oi < bi)) {
        bd = od;
        bi = oi;
    }
}

// Wave-cooperative exact nearest-point search for one sample (every lane
// holds the same sample).  On return (bd, bi) is the lexicographic minimum
// (squared distance, point row) over all points with distance^2 <= the
// initial bd, unless `retire` is set and the bound fell below M (then the
// function returns true early and (bd, bi) is only an upper bound).  With
// kIdx false only bd is kept (the flooding search needs the distance alone)
// and bi is left as it was.
// s_p0 / s_end: 64 entries of LDS per wave.
template <bool kIdx>
__device__ bool ring_search(const GridParam &g, const uint32_t *__restrict__ cs, const uint32_t *__restrict__ occ,
                            const float4 *__restrict__ xs,
                            float sx, float sy, float sz, float &bd, int32_t &bi, bool retire, float &M,
                            const uint64_t *__restrict__ keyj, uint32_t *s_p0, uint32_t *s_end, int lane,
                            unsigned long long &nev, uint32_t &steps) {
    if (retire && sqrt_rn(bd) < M) return true;
    const int cy = cell_of(sy, g.oy, g.inv_h, g.ny), cz = cell_of(sz, g.oz, g.inv_h, g.nz);
    const int rmax = max(max(cy, g.ny - 1 - cy), max(cz, g.nz - 1 - cz));
    const float h = g.h, eps = g.eps;
    for (int base = 0; ; base += 64) {
        int r0, dy0, dz0;
        ring_pos(base, r0, dy0, dz0);
        if (r0 > rmax) break;
        const float lbr = fmaxf((float)(r0 - 1) * h - eps, 0.f);
        if (lbr * lbr > bd) break;
        int r, dy, dz;
        ring_pos(base + lane, r, dy, dz);
        const int y = cy + dy, z = cz + dz;
        uint32_t p0 = 0, cnt = 0;
        if (r <= rmax && y >= 0 && y < g.ny && z >= 0 && z < g.nz) {
            const float ez = fmaxf(fmaxf((g.oz + (float)z * h - eps) - sz, sz - (g.oz + (float)(z + 1) * h + eps)), 0.f);
            const float ey = fmaxf(fmaxf((g.oy + (float)y * h - eps) - sy, sy - (g.oy + (float)(y + 1) * h + eps)), 0.f);
            const float lzy = ez * ez + ey * ey;
            if (!(lzy > bd)) {
                const float w = sqrtf(fmaxf(bd - lzy, 0.f)) + eps;
                const int x0 = cell_of(sx - w, g.ox, g.inv_h, g.nx);
                const int x1 = cell_of(sx + w, g.ox, g.inv_h, g.nx);
                const int64_t c0 = g.cell_base + ((int64_t)z * g.ny + y) * g.nx;
                if (any_occupied(occ, c0 + x0, c0 + x1)) {  // the offsets only for a run that holds points
                    p0 = cs[c0 + x0];
                    cnt = cs[c0 + x1 + 1] - p0;
                }
            }
        }
        // flatten the 64 rows' points; each lane takes kU consecutive ones
        const uint32_t incl = wave_incl_sum(cnt);
        const uint32_t total = rd_lane(incl, 63);
        s_p0[lane] = p0;
        s_end[lane] = incl;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        float lbd = bd;
        int32_t lbi = bi;
        if (lane == 0) nev += total;
        ++steps;
        for (uint32_t k0 = (uint32_t)lane * kU; k0 < total; k0 += 64 * kU) {
            int rr = 0;  // first row whose inclusive end exceeds k0 (six fixed steps)
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) rr += s_end[rr + st - 1] <= k0 ? st : 0;
            uint32_t pp[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t kk = k0 + u;
                pp[u] = 0xffffffffu;
                if (kk < total) {
                    while (s_end[rr] <= kk) ++rr;
                    pp[u] = s_p0[rr] + (kk - (rr ? s_end[rr - 1] : 0u));
                }
            }
            float4 cc[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (pp[u] != 0xffffffffu) cc[u] = xs[pp[u]];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (pp[u] != 0xffffffffu) {
                    const float d2 = dist2(sx, sy, sz, cc[u].x, cc[u].y, cc[u].z);
                    if (kIdx) lex_min(lbd, lbi, d2, __float_as_int(cc[u].w));
                    else lbd = fminf(lbd, d2);
                }
        }
        __builtin_amdgcn_wave_barrier();
        if (kIdx) {
            uint32_t mmin;  // distances are non-negative: float order is bit order
            const int src = wave_argmin_pair(__float_as_uint(lbd), (uint32_t)lbi, mmin);
            bd = __uint_as_float(mmin);
            bi = (int32_t)rd_lane((uint32_t)lbi, src);
        } else {
            bd = wave_min_f32_dpp(lbd);
        }
        if (retire) {
            if ((base & 511) == 448)
                M = fmaxf(M, key_value(__hip_atomic_load(keyj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
            if (sqrt_rn(bd) < M) return true;
        }
    }
    return false;
}

__device__ __forceinline__ int find_cloud(const int64_t *__restrict__ s_off, int32_t B, int64_t j) {
    int lo_b = 0, hi_b = B;
    while (hi_b - lo_b > 1) {
        const int mid = (lo_b + hi_b) >> 1;
        if (s_off[mid] <= j) lo_b = mid;
        else hi_b = mid;
    }
    return lo_b;
}

static constexpr uint32_t kGrab = 4;       // queue entries a wave takes per atomic on long queues
static constexpr uint32_t kGrabSmall = 1;  // on short queues (tail balance)
// The queue is read through kQueues cursors, each on a 256-byte line of its
// own: atomics on one line are serialised, so a single line shared by every
// wave caps the rate at which waves can take work.  Cursor c takes the
// segments c, c + kQueues, ... of kSeg entries (neighbouring open samples
// come from one tile); workgroup b reads through cursor b mod kQueues.
static constexpr uint32_t kQueues = 16;
static constexpr uint32_t kCursorStride = 64;  // uint32 words between cursors
static constexpr uint32_t kSeg = 16;

// queue position of the v-th entry taken through cursor c (increases with v)
__device__ __forceinline__ uint32_t seg_index(uint32_t v, uint32_t c) {
    return ((v / kSeg) * kQueues + c) * kSeg + v % kSeg;
}

__global__ __launch_bounds__(kWaveBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_flood_deep(
    DeepArgs a, const float *__restrict__ seed, uint64_t *__restrict__ key, const GridParam *__restrict__ gp,
    const uint32_t *__restrict__ cs, const uint32_t *__restrict__ occ, const float4 *__restrict__ xs,
    OpenSample *__restrict__ queue,
    const uint32_t *__restrict__ queue_count, uint32_t *__restrict__ queue_next,
    unsigned long long *__restrict__ evals, unsigned long long *__restrict__ stats) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ uint32_t s_p0[kWaveBlock / 64][64], s_end[kWaveBlock / 64][64];
    const uint32_t n = *queue_count;
    if (stats && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&stats[4 * a.d + 1], (unsigned long long)n);
    unsigned long long nev = 0;
    uint32_t nsteps = 0;  // ring steps (64 rows each) of this wave
    uint32_t wmax_steps = 0, wlong = 0;  // its longest search; its searches of more than 32 steps
    const uint32_t cur = blockIdx.x % kQueues;
    const uint32_t grab = a.grab ? a.grab : (n > (1u << 19) ? kGrab : kGrabSmall);
    while (true) {
        uint32_t v0 = 0;
        if (lane == 0) v0 = atomicAdd(&queue_next[cur * kCursorStride], grab);
        v0 = __builtin_amdgcn_readfirstlane(v0);
        if (seg_index(v0, cur) >= n) break;
        // lanes 0..grab-1 fetch the grabbed entries and their simplices'
        // running values together (a stale value only retires less)
        float4 qp = make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t qg = 0, qc = 0;
        float qm = 0.f;
        if (lane < (int)grab) {
            const uint32_t i = seg_index(v0 + lane, cur);
            if (i < n) {
                const OpenSample o = queue[i];
                qp = o.p;
                qg = o.gid;
                qc = o.cloud;
                const uint32_t j = o.gid / (uint32_t)a.n_int;
                qm = fmaxf(seed[j], key_value(__hip_atomic_load(&key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
            }
        }
        for (int u = 0; u < (int)grab; ++u) {
            if (seg_index(v0 + u, cur) >= n) break;
            const float sx = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(qp.x), u));
            const float sy = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(qp.y), u));
            const float sz = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(qp.z), u));
            float bd = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(qp.w), u));
            float M = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(qm), u));
            const uint32_t gid = __builtin_amdgcn_readlane(qg, u);
            const GridParam g = gp[__builtin_amdgcn_readlane(qc, u)];
            const int64_t j = gid / (uint32_t)a.n_int;
            const int q = (int)(gid % (uint32_t)a.n_int);
            int32_t bi = 0x7fffffff;
            const uint32_t steps0 = nsteps;
            // the point row is kept as well: when this sample wins, its x*
            // is this search's (the same lexicographic minimum the winner
            // search would find), and that search is skipped
            const bool retired = ring_search<true>(g, cs, occ, xs, sx, sy, sz, bd, bi, a.d > 0, M, &key[j],
                                                   s_p0[wid], s_end[wid], lane, nev, nsteps);
            wmax_steps = max(wmax_steps, nsteps - steps0);
            wlong += nsteps - steps0 > 32 ? 1u : 0u;
            if (lane == 0) {
                const uint32_t i = seg_index(v0 + u, cur);
                if (!retired) publish(key, seed, (int32_t)j, q, bd, a.d == 0, a.sampling == FLOOD_SAMPLING_RANDOM);
                queue[i].xrow = retired || bi == 0x7fffffff ? kNoRow : (uint32_t)bi;
                queue[i].val = __float_as_uint(sqrt_rn(bd));
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nev += __shfl_xor(nev, o, 64);
    if (evals && lane == 0 && nev) atomicAdd(evals, nev);
    if (stats && lane == 0 && nev) atomicAdd(&stats[4 * a.d + 3], nev);
    if (stats && lane == 0 && nsteps) atomicAdd(&stats[4 * a.d], (unsigned long long)nsteps);
    if (stats && lane == 0 && wmax_steps) atomicMax(&stats[16 + 4 * a.d + 1], (unsigned long long)wmax_steps);
    if (stats && lane == 0 && wlong) atomicAdd(&stats[16 + 4 * a.d + 2], (unsigned long long)wlong);
}

// winners whose sample the per-sample search completed: x* is that search's
// nearest point; the key is cleared so the winner search skips the simplex
// (after k_winner, which reads the key)
__global__ __launch_bounds__(256) void k_match_winners(const OpenSample *__restrict__ queue,
                                                       const uint32_t *__restrict__ queue_count, int32_t n_int,
                                                       uint64_t *__restrict__ key, int32_t *__restrict__ win_x) {
    const uint32_t n = *queue_count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const OpenSample o = queue[i];
        if (o.xrow == kNoRow) continue;
        const uint32_t j = o.gid / (uint32_t)n_int, q = o.gid % (uint32_t)n_int;
        if (key[j] == (((uint64_t)o.val << 32) | (uint64_t)(0xffffffffu - q))) {
            win_x[j] = (int32_t)o.xrow;
            key[j] = 0;
        }
    }
}

// simplices still needing x* (an own sample won and no per-sample search
// gave its point): a list in kQueues regions, region c filled by the
// workgroups b = c mod kQueues (so its size is bounded by the simplices those
// workgroups cover, cap each), one atomic per wavefront on the region's count
__host__ __device__ __forceinline__ int64_t winner_region_cap(int64_t n) {
    return ((n + 255) / 256 + kQueues - 1) / kQueues * 256;
}
__global__ __launch_bounds__(256) void k_winner_list(int64_t n, int32_t B, const int64_t *__restrict__ s_off,
                                                     const uint64_t *__restrict__ key, uint32_t *__restrict__ wcount,
                                                     uint32_t *__restrict__ wlist, uint32_t *__restrict__ wcloud) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool need = j < n && key[j] != 0;
    const uint64_t m = __ballot(need);
    if (!m) return;
    const uint32_t c = blockIdx.x % kQueues;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&wcount[c * kCursorStride], (uint32_t)__popcll(m));
    base = __shfl(base, 0, 64);
    if (need) {
        const int64_t at = c * winner_region_cap(n) + base + __popcll(m & ((1ull << lane) - 1ull));
        wlist[at] = (uint32_t)j;
        wcloud[at] = (uint32_t)find_cloud(s_off, B, j);
    }
}

// x* of the winning own sample of the listed simplices: persistent
// wavefronts take list entries through the region cursors; the value is
// known, so the search ball is exact and tiny for most simplices
__global__ __launch_bounds__(kWaveBlock) void k_winner_search(
    int64_t n, int32_t n_int, const float4 *__restrict__ spos, const uint64_t *__restrict__ key,
    const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs, const uint32_t *__restrict__ occ,
    const float4 *__restrict__ xs, const uint32_t *__restrict__ wcount, uint32_t *__restrict__ wnext,
    const uint32_t *__restrict__ wlist, const uint32_t *__restrict__ wcloud, int32_t *__restrict__ win_x) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __shared__ uint32_t s_p0[kWaveBlock / 64][64], s_end[kWaveBlock / 64][64];
    const uint32_t c = blockIdx.x % kQueues;
    const uint32_t cnt = wcount[c * kCursorStride];
    const uint32_t grab = cnt > (1u << 15) ? kGrab : 1u;
    const uint32_t *list = wlist + c * winner_region_cap(n), *lcloud = wcloud + c * winner_region_cap(n);
    while (true) {
        uint32_t v0 = 0;
        if (lane == 0) v0 = atomicAdd(&wnext[c * kCursorStride], grab);
        v0 = __builtin_amdgcn_readfirstlane(v0);
        if (v0 >= cnt) break;
        for (uint32_t u = 0; u < grab && v0 + u < cnt; ++u) {
            const int64_t j = __builtin_amdgcn_readfirstlane(list[v0 + u]);
            const int b = (int)__builtin_amdgcn_readfirstlane(lcloud[v0 + u]);
            const uint64_t kv = key[j];
            const int q = (int)(0xffffffffu - (uint32_t)(kv & 0xffffffffu));
            // the winning sample's point, as the sample sort computed it
            const float4 sp = spos[j * n_int + q];
            const float sx = sp.x, sy = sp.y, sz = sp.z;
            const float val = key_value(kv);
            const float rb = val * (1.0f + 1e-6f) + 1e-30f;
            float bd = rb * rb;
            int32_t bi = 0x7fffffff;
            float M = 0.f;
            unsigned long long nev = 0;
            uint32_t nsteps = 0;
            const GridParam g = gp[b];
            ring_search<true>(g, cs, occ, xs, sx, sy, sz, bd, bi, false, M, nullptr, s_p0[wid], s_end[wid], lane, nev,
                              nsteps);
            if (lane == 0) win_x[j] = bi;
        }
    }
}

// ---------------------------------------------------------------------------
// winner record and final value: one thread per simplex.  An own sample won
// if the key is set (x* was written by phase B); otherwise the value is the
// seed and the winner is inherited from the first facet attaining it.

__device__ __forceinline__ uint32_t pack_comp(const int a[4]) {
    return (uint32_t)a[0] | ((uint32_t)a[1] << 8) | ((uint32_t)a[2] << 16) | ((uint32_t)a[3] << 24);
}

__global__ void k_winner(int d, SampleRule rule, int64_t n, int32_t B, const int64_t *__restrict__ s_off,
                         const int32_t *__restrict__ simp,
                         const int32_t *__restrict__ tri_edges, const int32_t *__restrict__ tet_tris,
                         const float *__restrict__ seed, const uint64_t *__restrict__ key, const float *__restrict__ fprev,
                         const int32_t *__restrict__ wxprev, const uint32_t *__restrict__ waprev,
                         const float *__restrict__ wwprev, float *__restrict__ f, int32_t *__restrict__ win_x,
                         uint32_t *__restrict__ win_a, float *__restrict__ win_w) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool random = rule.sampling == FLOOD_SAMPLING_RANDOM;
    const uint64_t kv = key[j];
    if (kv != 0) {
        const int q = (int)(0xffffffffu - (uint32_t)(kv & 0xffffffffu));
        f[j] = key_value(kv);  // win_x comes from k_winner_search
        if (random) {
            win_a[j] = (uint32_t)q | (((1u << (d + 1)) - 1u) << 28);
        } else {
            int comp[4] = {0, 0, 0, 0};
            if (d == 0) comp[0] = rule.k;
            else unrank_interior(q, d, rule.k, comp);
            win_a[j] = pack_comp(comp);
        }
        if (win_w) {
            float w[4];
            own_weights(rule, d, q, j - s_off[find_cloud(s_off, B, j)], w);
            *(float4 *)&win_w[4 * j] = make_float4(w[0], w[1], w[2], w[3]);
        }
        return;
    }
    const float sd = seed[j];
    int32_t fac[4];
    for (int i = 0; i <= d; ++i) {
        if (d == 1) fac[i] = simp[2 * j + (1 - i)];
        else if (d == 2) fac[i] = tri_edges[3 * j + i];
        else fac[i] = tet_tris[4 * j + i];
    }
    int fi = 0;
    for (int i = 0; i <= d; ++i)
        if (fprev[fac[i]] == sd) { fi = i; break; }
    const uint32_t pa = waprev[fac[fi]];
    f[j] = sd;
    win_x[j] = wxprev[fac[fi]];
    if (random) {
        // the owner's vertex set: the facet's bits with vertex fi left out
        const uint32_t m = pa >> 28, lowm = (1u << fi) - 1u;
        win_a[j] = (pa & 0x0fffffffu) | (((m & lowm) | ((m & ~lowm) << 1)) << 28);
    } else {
        const int fa[4] = {(int)(pa & 255), (int)((pa >> 8) & 255), (int)((pa >> 16) & 255), (int)(pa >> 24)};
        int aa[4] = {0, 0, 0, 0};
        for (int i = 0, src = 0; i <= d; ++i) aa[i] = (i == fi) ? 0 : fa[src++];
        win_a[j] = pack_comp(aa);
    }
    if (win_w) {
        const float4 pw = *(const float4 *)&wwprev[4 * (int64_t)fac[fi]];
        const float fw[4] = {pw.x, pw.y, pw.z, pw.w};
        float ww[4] = {0.f, 0.f, 0.f, 0.f};
        for (int i = 0, src = 0; i <= d; ++i) ww[i] = (i == fi) ? 0.f : fw[src++];
        *(float4 *)&win_w[4 * j] = make_float4(ww[0], ww[1], ww[2], ww[3]);
    }
}

// ---------------------------------------------------------------------------
// host driver

size_t flood_workspace(const flood_problem *pb, float alpha, FloodSizes *sz) {
    int64_t tc = 0;
    size_t bytes = grid_workspace(pb->B, pb->x_off, alpha, &tc);
    int64_t n[4];
    n[0] = pb->l_off[pb->B];
    int64_t nmax = n[0];
    for (int d = 1; d < 4; ++d) {
        n[d] = pb->s_off[d][pb->B];
        nmax = n[d] > nmax ? n[d] : nmax;
    }
    int64_t smax = 0;
    for (int d = 0; d < 4; ++d) {
        int64_t sm = n[d] * own_samples(d, pb->k, pb->sampling);
        smax = sm > smax ? sm : smax;
    }
    bytes += sizeof(float) * (nmax + 1) + 256;        // seed
    bytes += sizeof(uint64_t) * (nmax + 1) + 256;     // key
    bytes += sizeof(OpenSample) * (smax + 1) + 256;   // open-sample queue
    int64_t bkmax = 0;
    for (int d = 0; d < 4; ++d) {
        int64_t bk = 0;
        const int64_t *so = d == 0 ? pb->l_off : pb->s_off[d];
        for (int32_t b = 0; b < pb->B; ++b) bk += (int64_t)1 << (3 * morton_bits((so[b + 1] - so[b]) * own_samples(d, pb->k, pb->sampling)));
        bkmax = bk > bkmax ? bk : bkmax;
    }
    bytes += 2 * (sizeof(uint32_t) * (smax + 1) + 256);  // sample keys and order
    bytes += sizeof(float4) * (smax + 1) + 256;           // sample points and bounds
    bytes += sizeof(uint32_t) * (bkmax + 1) + 256;       // bucket counts (then starts)
    bytes += sizeof(uint32_t) * (smax + 1) + 256;        // sample ranks within their buckets
    bytes += sizeof(uint32_t) * 2 * kCursorStride * kQueues + 256;  // winner list counts and cursors
    bytes += 2 * (sizeof(uint32_t) * kQueues * winner_region_cap(nmax) + 256);  // winner list and clouds
    bytes += sizeof(uint32_t) * scan_tmp_elems(bkmax + 1) + 256;
    bytes += sizeof(int32_t) * (pb->B + 1) + sizeof(uint32_t) * (pb->B + 1) + 512;
    bytes += sizeof(uint32_t) * kCursorStride * (kQueues + 1) + 256;  // queue count and cursors
    bytes += 4 * (sizeof(int64_t) * (pb->B + 1) + 256); // tile offsets
    bytes += sizeof(uint32_t) * (smax / 16 + pb->B + 1) + 256;  // the cloud of every tile
    bytes += sizeof(uint32_t) * (nmax + 1) + 256;                // the cloud of every simplex
    bytes += 1024;
    if (sz) {
        for (int d = 0; d < 4; ++d) sz->n[d] = n[d];
        sz->total_pts = pb->x_off[pb->B];
        sz->total_cells = tc;
    }
    return bytes;
}

template <int T>
static void launch_tiles(const TileArgs &ta, int wpb, hipStream_t s, const float4 *spos,
                         const int64_t *s_off, const int64_t *tile_off, const uint32_t *tcloud, const float *seed,
                         uint64_t *key,
                         const GridWork &g, const uint32_t *order, OpenSample *hard, uint32_t *hard_count,
                         uint64_t *evals, uint64_t *stats) {
    const int64_t nb = (ta.n_tiles + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_flood_tiles<T>, dim3((unsigned)nb), dim3(64 * wpb), 0, s, ta, spos, s_off, tile_off,
                       tcloud, seed, key, g.gp, g.cell_start, g.xs, order, hard, hard_count, (unsigned long long *)evals,
                       (unsigned long long *)stats);
}

hipError_t flood_run(const flood_problem *pb, const flood_tuning &tu, const flood_outputs *out, void *ws,
                     size_t ws_bytes, hipStream_t s) {
    FloodSizes sz;
    flood_workspace(pb, tu.cells_per_point, &sz);
    Carve c(ws, ws_bytes);
    GridWork g;
    grid_carve(c, pb->B, pb->x_off, tu.cells_per_point, g);
    int64_t nmax = 0;
    for (int d = 0; d < 4; ++d) nmax = sz.n[d] > nmax ? sz.n[d] : nmax;
    int64_t smax = 0;
    for (int d = 0; d < 4; ++d) {
        int64_t sm = sz.n[d] * own_samples(d, pb->k, pb->sampling);
        smax = sm > smax ? sm : smax;
    }
    float *seed = c.take<float>(nmax + 1);
    uint64_t *key = c.take<uint64_t>(nmax + 1);
    OpenSample *hard = c.take<OpenSample>(smax + 1);
    // [0] open samples; the queue cursors from word kCursorStride on, kCursorStride apart
    uint32_t *counters = c.take<uint32_t>(kCursorStride * (kQueues + 1));
    int64_t bkmax = 0;
    for (int d = 0; d < 4; ++d) {
        int64_t bk = 0;
        const int64_t *so = d == 0 ? pb->l_off : pb->s_off[d];
        for (int32_t b = 0; b < pb->B; ++b) bk += (int64_t)1 << (3 * morton_bits((so[b + 1] - so[b]) * own_samples(d, pb->k, pb->sampling)));
        bkmax = bk > bkmax ? bk : bkmax;
    }
    uint32_t *skey = c.take<uint32_t>(smax + 1);
    uint32_t *order = c.take<uint32_t>(smax + 1);
    float4 *spos = c.take<float4>(smax + 1);  // sample points and bounds, in global sample order
    uint32_t *bcount = c.take<uint32_t>(bkmax + 1);
    uint32_t *srank = c.take<uint32_t>(smax + 1);
    // the winner search's list: region counts, then region cursors (kCursorStride apart); the list
    uint32_t *wcounters = c.take<uint32_t>(2 * kCursorStride * kQueues);
    uint32_t *wlist = c.take<uint32_t>(kQueues * winner_region_cap(nmax));
    uint32_t *wcloud = c.take<uint32_t>(kQueues * winner_region_cap(nmax));  // the listed simplices' clouds
    uint32_t *bscan = c.take<uint32_t>(scan_tmp_elems(bkmax + 1));
    int32_t *mbits = c.take<int32_t>(pb->B + 1);
    uint32_t *bbase = c.take<uint32_t>(pb->B + 1);
    int64_t *tile_off[4];
    for (int d = 0; d < 4; ++d) tile_off[d] = c.take<int64_t>(pb->B + 1);
    uint32_t *tcloud = c.take<uint32_t>(smax / 16 + pb->B + 1);  // tiles have at least 16 samples
    uint32_t *scloud = c.take<uint32_t>(nmax + 1);                // the cloud of every simplex
    if (!c.ok()) return hipErrorOutOfMemory;

    hipError_t e = hipSuccess;
    if (out->grid_events[0] && (e = hipEventRecord((hipEvent_t)out->grid_events[0], s)) != hipSuccess) return e;
    e = grid_build(pb->X, pb->B, pb->x_off, pb->x_off_d, tu.cells_per_point, g, s);
    if (e != hipSuccess) return e;
    if (out->grid_events[1] && (e = hipEventRecord((hipEvent_t)out->grid_events[1], s)) != hipSuccess) return e;
    const int T = tu.samples_per_lane;
    const int wpb = tu.waves_per_block;
    // samples per tile by dimension (T = 1): one value from the tuning, or
    // the defaults below
    int tile_lanes[4];
    for (int d = 0; d < 4; ++d) tile_lanes[d] = tu.tile_lanes ? tu.tile_lanes : kTileLanesDefault[d];
    for (int d = 0; d < 4; ++d) {
        const int64_t n = sz.n[d];
        if (n == 0) continue;
        const int64_t nint = own_samples(d, pb->k, pb->sampling);
        const SampleRule rule{pb->k, pb->sampling, pb->seed};
        const int64_t *soff_h = d == 0 ? pb->l_off : pb->s_off[d];
        const int64_t *soff_d = d == 0 ? pb->l_off_d : pb->s_off_d[d];
        const int32_t *simp = d == 0 ? nullptr : pb->simp[d];
        hipLaunchKernelGGL(k_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n, pb->simp[1],
                           pb->tri_edges, pb->tet_tris, d > 0 ? out->f[d - 1] : nullptr, seed);
        e = fill_u64(key, 0ull, n, s);
        if (e != hipSuccess) return e;
        e = fill_u32(counters, 0u, kCursorStride * (kQueues + 1), s);
        if (e != hipSuccess) return e;
        int64_t ntiles_d = 0;  // tiles of this dimension (0: no search ran)
        if (nint > 0) {
            const int64_t tsamp = (T == 1 ? (int64_t)tile_lanes[d] : 64) * (int64_t)T;
            int64_t ntiles = 0;
            for (int32_t b = 0; b < pb->B; ++b) ntiles += ((soff_h[b + 1] - soff_h[b]) * nint + tsamp - 1) / tsamp;
            ntiles_d = ntiles;
            hipLaunchKernelGGL(k_tile_off, dim3(1), dim3(1024), 0, s, soff_d, pb->B, nint, tsamp, tile_off[d]);
            if (pb->B > 1 && ntiles > 0)
                hipLaunchKernelGGL(k_tile_cloud, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, tile_off[d],
                                   pb->B, ntiles, tcloud);
            // spatial order of the samples
            int64_t bk = 0;
            for (int32_t b = 0; b < pb->B; ++b) bk += (int64_t)1 << (3 * morton_bits((soff_h[b + 1] - soff_h[b]) * nint));
            const int64_t S = n * nint;
            hipLaunchKernelGGL(k_bucket_base, dim3(1), dim3(1024), 0, s, soff_d, pb->B, nint, mbits, bbase);
            e = fill_u32(bcount, 0u, bk + 1, s);
            if (e != hipSuccess) return e;
            if (pb->B > 1)
                hipLaunchKernelGGL(k_simplex_cloud, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, soff_d, pb->B, n,
                                   scloud);
            hipLaunchKernelGGL(k_sample_keys, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, d, rule, (int)nint,
                               pb->B, S, pb->Lxyz, simp, soff_d, scloud, g.gp, mbits, bbase, pb->X, pb->l_xidx,
                               pb->x_off_d, pb->landmarks_in_x, skey, srank, bcount, spos);
            e = exclusive_scan_u32(bcount, bk + 1, bscan, s);  // bucket starts
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_sample_scatter, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, s, S, skey, srank,
                               bcount, order);
            if (ntiles > 0) {
                TileArgs ta;
                ta.d = d;
                ta.k = pb->k;
                ta.n_int = (int32_t)nint;
                ta.landmarks_in_x = pb->landmarks_in_x;
                ta.B = pb->B;
                ta.radius_budget = tu.tile_shells - 1;  // -2 disables the cooperative phase
                ta.max_extent = tu.tile_extent;
                ta.sampling = pb->sampling;
                ta.n_tiles = ntiles;
                ta.seed = pb->seed;
                ta.lanes = T == 1 ? tile_lanes[d] : 64;
                ta.pad = 0;
                if (out->tile_events[3 * d]) {
                    e = hipEventRecord((hipEvent_t)out->tile_events[3 * d], s);
                    if (e != hipSuccess) return e;
                }
                if (T == 1) launch_tiles<1>(ta, wpb, s, spos, soff_d, tile_off[d], tcloud, seed, key, g, order, hard, counters, out->evals, out->stats);
                else if (T == 2) launch_tiles<2>(ta, wpb, s, spos, soff_d, tile_off[d], tcloud, seed, key, g, order, hard, counters, out->evals, out->stats);
                else launch_tiles<4>(ta, wpb, s, spos, soff_d, tile_off[d], tcloud, seed, key, g, order, hard, counters, out->evals, out->stats);
                if (out->tile_events[3 * d + 1]) {
                    e = hipEventRecord((hipEvent_t)out->tile_events[3 * d + 1], s);
                    if (e != hipSuccess) return e;
                }
                DeepArgs da;
                da.d = d;
                da.k = pb->k;
                da.n_int = (int32_t)nint;
                da.B = pb->B;
                da.grab = (uint32_t)tu.queue_grab;
                da.sampling = pb->sampling;
                hipLaunchKernelGGL(k_flood_deep, dim3(2048), dim3(256), 0, s, da, seed, key,
                                   g.gp, g.cell_start, g.occ, g.xs, hard, counters, counters + kCursorStride,
                                   (unsigned long long *)out->evals, (unsigned long long *)out->stats);
                if (out->tile_events[3 * d + 2]) {
                    e = hipEventRecord((hipEvent_t)out->tile_events[3 * d + 2], s);
                    if (e != hipSuccess) return e;
                }
            }
        }
        hipLaunchKernelGGL(k_winner, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, rule, n, pb->B, soff_d,
                           simp, pb->tri_edges, pb->tet_tris, seed, key, d > 0 ? out->f[d - 1] : nullptr,
                           d > 0 ? out->win_x[d - 1] : nullptr, d > 0 ? out->win_a[d - 1] : nullptr,
                           d > 0 ? out->win_w[d - 1] : nullptr, out->f[d], out->win_x[d], out->win_a[d],
                           out->win_w[d]);
        if (nint > 0 && ntiles_d > 0)
            hipLaunchKernelGGL(k_match_winners, dim3(1024), dim3(256), 0, s, hard, counters, (int32_t)nint, key,
                               out->win_x[d]);
        e = fill_u32(wcounters, 0u, 2 * kCursorStride * kQueues, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_winner_list, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, pb->B, soff_d, key,
                           wcounters, wlist, wcloud);
        hipLaunchKernelGGL(k_winner_search, dim3(2048), dim3(256), 0, s, n, (int32_t)nint, spos, key, g.gp,
                           g.cell_start, g.occ, g.xs, wcounters, wcounters + kCursorStride * kQueues, wlist, wcloud,
                           out->win_x[d]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace flood
