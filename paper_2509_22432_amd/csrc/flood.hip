// The flooding step: for every simplex sigma of Del(L), the sampled flood
// value f(sigma) = max_{tau face of sigma} max_{p in P_tau} min_{x in X} ||p-x||
// (Def. 1, Sec. 4.1; P_tau the barycentric grid of Lemma 6, k segments per
// edge).  Dimensions run bottom-up.  A simplex only evaluates its INTERIOR
// samples (all a_i >= 1): the samples on its boundary belong to its facets,
// whose values arrive as the seed M = max over facets f(tau) -- the closure
// of Sec. 4.1, and exactly the max over the full grid because P_tau is a
// subset of P_sigma.
//
// Search (one wavefront per tile of 64*T consecutive samples; consecutive
// simplices share their first vertex, so a tile is spatially compact):
//  * each sample starts from the bound d(p,X)^2 <= min_i |p - v_i|^2, valid
//    when the landmarks are points of X (proof of Lemma 7);
//  * the wave scans grid cells in growing boxes around its samples, one
//    x-run of cells (contiguous points) at a time; a run is skipped unless
//    some live sample's distance to the run's box is below its bound; the
//    points of a run are read at wave-uniform addresses (scalar loads) and
//    every live lane updates its minimum with direct-difference FP32;
//  * a sample retires as soon as its bound drops below the simplex's
//    running max M (it cannot raise f), and completes when its bound is
//    below the distance to the unscanned region (its minimum is exact);
//  * completed samples above the seed publish (value, rank) with a 64-bit
//    atomic max per simplex, which other tiles read to raise M.
// Every skip is conservative, so the result equals the unpruned max-min.
#include "sample.hpp"

namespace flood {

static constexpr int kWaveBlock = 256;

// ---------------------------------------------------------------------------
// per-dimension helpers

// tile offsets per cloud: tiles_b = ceil(n_b * n_int / (64 T))
__global__ void k_tile_off(const int64_t *s_off, int32_t B, int64_t n_int, int64_t tile_samples, int64_t *tile_off) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t t = 0;
    for (int32_t b = 0; b < B; ++b) {
        tile_off[b] = t;
        int64_t S = (s_off[b + 1] - s_off[b]) * n_int;
        t += (S + tile_samples - 1) / tile_samples;
    }
    tile_off[B] = t;
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
// the tile kernel

struct TileArgs {
    int32_t d, k, n_int, landmarks_in_x;
    int32_t B, pad;
    int64_t n_tiles;
};

template <int T>
__global__ __launch_bounds__(kWaveBlock) void k_flood_tiles(
    TileArgs a, const float *__restrict__ L, const int32_t *__restrict__ lxidx, const int32_t *__restrict__ simp,
    const int64_t *__restrict__ s_off, const int64_t *__restrict__ tile_off, const float *__restrict__ seed,
    uint64_t *__restrict__ key, const GridParam *__restrict__ gp, const uint32_t *__restrict__ cs,
    const float4 *__restrict__ xs, unsigned long long *__restrict__ evals) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    // wave-uniform by construction; readfirstlane lets the compiler keep the
    // tile state in scalar registers and load points with scalar loads
    const int64_t wave = xcd_remap(blockIdx.x, gridDim.x) * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= a.n_tiles) return;
    int lo_b = 0, hi_b = a.B;
    while (hi_b - lo_b > 1) {
        int mid = (lo_b + hi_b) >> 1;
        if (tile_off[mid] <= wave) lo_b = mid;
        else hi_b = mid;
    }
    const int b = lo_b;
    const GridParam g = gp[b];
    const int64_t sbase = s_off[b];
    const int64_t S = (s_off[b + 1] - sbase) * (int64_t)a.n_int;
    const int64_t ls0 = (wave - tile_off[b]) * 64 * T;
    const int d = a.d;

    float sx[T], sy[T], sz[T], best[T], M[T];
    int32_t sj[T], sq[T];
    bool valid[T], live[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int64_t ls = ls0 + (int64_t)t * 64 + lane;
        valid[t] = ls < S;
        sx[t] = sy[t] = sz[t] = 0.f;
        best[t] = 0.f;
        M[t] = 0.f;
        sj[t] = 0;
        sq[t] = 0;
        if (valid[t]) {
            const int64_t j = sbase + ls / a.n_int;
            const int q = (int)(ls % a.n_int);
            sj[t] = (int32_t)j;
            sq[t] = q;
            int comp[4];
            if (d == 0) {
                comp[0] = a.k;
            } else {
                unrank_interior(q, d, a.k, comp);
            }
            int32_t v[4];
            simplex_vertices(simp, d, j, v);
            sample_point(L, v, comp, d, a.k, sx[t], sy[t], sz[t]);
            float u = INFINITY;
            if (a.landmarks_in_x) {
                for (int i = 0; i <= d; ++i)
                    u = fminf(u, dist2(sx[t], sy[t], sz[t], L[3 * v[i]], L[3 * v[i] + 1], L[3 * v[i] + 2]));
            }
            best[t] = u;
            M[t] = seed[j];
        }
        live[t] = valid[t] && !(__fsqrt_rn(best[t]) < M[t]);
    }

    // initial box: the cells of the live samples
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    bool any = false;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (live[t]) {
            const int cx = cell_of(sx[t], g.ox, g.inv_h, g.nx);
            const int cy = cell_of(sy[t], g.oy, g.inv_h, g.ny);
            const int cz = cell_of(sz[t], g.oz, g.inv_h, g.nz);
            lo[0] = min(lo[0], cx); hi[0] = max(hi[0], cx);
            lo[1] = min(lo[1], cy); hi[1] = max(hi[1], cy);
            lo[2] = min(lo[2], cz); hi[2] = max(hi[2], cz);
            any = true;
        }
    }
    unsigned long long nev = 0;
    if (__any(any)) {
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
        int olo[3] = {lo[0], lo[1], lo[2]}, ohi[3] = {lo[0] - 1, lo[1] - 1, lo[2] - 1};  // empty old box
        bool first = true;
        const float h = g.h, eps = g.eps;
        while (true) {
            // scan the rows of box [lo,hi] minus box [olo,ohi]
            for (int z = lo[2]; z <= hi[2]; ++z) {
                for (int y = lo[1]; y <= hi[1]; ++y) {
                    const bool inner = !first && z >= olo[2] && z <= ohi[2] && y >= olo[1] && y <= ohi[1];
                    for (int part = 0; part < 2; ++part) {
                        int x0, x1;
                        if (!inner) {
                            if (part) break;
                            x0 = lo[0];
                            x1 = hi[0];
                        } else if (part == 0) {
                            x0 = lo[0];
                            x1 = olo[0] - 1;
                        } else {
                            x0 = ohi[0] + 1;
                            x1 = hi[0];
                        }
                        if (x0 > x1) continue;
                        const int64_t c0 = g.cell_base + ((int64_t)z * g.ny + y) * g.nx + x0;
                        const uint32_t p0 = __builtin_amdgcn_readfirstlane(cs[c0]);
                        const uint32_t p1 = __builtin_amdgcn_readfirstlane(cs[c0 + (x1 - x0) + 1]);
                        if (p0 == p1) continue;
                        // conservative box of the run
                        const float bx0 = g.ox + (float)x0 * h - eps, bx1 = g.ox + (float)(x1 + 1) * h + eps;
                        const float by0 = g.oy + (float)y * h - eps, by1 = g.oy + (float)(y + 1) * h + eps;
                        const float bz0 = g.oz + (float)z * h - eps, bz1 = g.oz + (float)(z + 1) * h + eps;
                        bool need = false;
                        int nlive = 0;
#pragma unroll
                        for (int t = 0; t < T; ++t) {
                            if (live[t]) {
                                const float ex = fmaxf(fmaxf(bx0 - sx[t], sx[t] - bx1), 0.f);
                                const float ey = fmaxf(fmaxf(by0 - sy[t], sy[t] - by1), 0.f);
                                const float ez = fmaxf(fmaxf(bz0 - sz[t], sz[t] - bz1), 0.f);
                                const float lb = ex * ex + ey * ey + ez * ez;
                                need |= lb < best[t];
                            }
                            nlive += __popcll(__ballot(live[t]));
                        }
                        if (!__any(need)) continue;
                        nev += (unsigned long long)(p1 - p0) * (unsigned long long)nlive;
                        uint32_t p = p0;
                        for (; p + 3 < p1; p += 4) {
                            const float4 q0 = xs[p], q1 = xs[p + 1], q2 = xs[p + 2], q3 = xs[p + 3];
#pragma unroll
                            for (int t = 0; t < T; ++t) {
                                const float d0 = dist2(sx[t], sy[t], sz[t], q0.x, q0.y, q0.z);
                                const float d1 = dist2(sx[t], sy[t], sz[t], q1.x, q1.y, q1.z);
                                const float d2 = dist2(sx[t], sy[t], sz[t], q2.x, q2.y, q2.z);
                                const float d3 = dist2(sx[t], sy[t], sz[t], q3.x, q3.y, q3.z);
                                best[t] = fminf(fminf(best[t], fminf(d0, d1)), fminf(d2, d3));
                            }
                        }
                        for (; p + 1 < p1; p += 2) {
                            const float4 q0 = xs[p];
                            const float4 q1 = xs[p + 1];
#pragma unroll
                            for (int t = 0; t < T; ++t) {
                                const float d0 = dist2(sx[t], sy[t], sz[t], q0.x, q0.y, q0.z);
                                const float d1 = dist2(sx[t], sy[t], sz[t], q1.x, q1.y, q1.z);
                                best[t] = fminf(best[t], fminf(d0, d1));
                            }
                        }
                        if (p < p1) {
                            const float4 q0 = xs[p];
#pragma unroll
                            for (int t = 0; t < T; ++t)
                                best[t] = fminf(best[t], dist2(sx[t], sy[t], sz[t], q0.x, q0.y, q0.z));
                        }
                    }
                }
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
                const uint64_t kv = __hip_atomic_load(&key[sj[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                M[t] = fmaxf(M[t], key_value(kv));
                const bool complete = full || (ext > 0.f && best[t] <= ext * ext);
                if (complete) {
                    const float v = __fsqrt_rn(best[t]);
                    if (v > seed[sj[t]]) {
                        const uint64_t nk = ((uint64_t)__float_as_uint(v) << 32) | (uint64_t)(0xffffffffu - (uint32_t)sq[t]);
                        atomicMax((unsigned long long *)&key[sj[t]], (unsigned long long)nk);
                    }
                    live[t] = false;
                } else if (__fsqrt_rn(best[t]) < M[t]) {
                    live[t] = false;
                }
                anylive |= live[t];
            }
            if (!__any(anylive) || full) break;
            for (int ax = 0; ax < 3; ++ax) {
                olo[ax] = lo[ax];
                ohi[ax] = hi[ax];
            }
            lo[0] = max(lo[0] - 1, 0); hi[0] = min(hi[0] + 1, g.nx - 1);
            lo[1] = max(lo[1] - 1, 0); hi[1] = min(hi[1] + 1, g.ny - 1);
            lo[2] = max(lo[2] - 1, 0); hi[2] = min(hi[2] + 1, g.nz - 1);
            first = false;
        }
    }
    if (evals && lane == 0 && nev) atomicAdd(evals, nev);
}

// ---------------------------------------------------------------------------
// winner record: one wave per simplex

__device__ __forceinline__ uint32_t pack_comp(const int a[4]) {
    return (uint32_t)a[0] | ((uint32_t)a[1] << 8) | ((uint32_t)a[2] << 16) | ((uint32_t)a[3] << 24);
}

__global__ __launch_bounds__(kWaveBlock) void k_winner(
    int d, int k, int64_t n, const float *__restrict__ L, const int32_t *__restrict__ simp,
    const int32_t *__restrict__ tri_edges, const int32_t *__restrict__ tet_tris, const int64_t *__restrict__ s_off,
    int32_t B, const float *__restrict__ seed, const uint64_t *__restrict__ key, const GridParam *__restrict__ gp,
    const uint32_t *__restrict__ cs, const float4 *__restrict__ xs, const float *__restrict__ fprev,
    const int32_t *__restrict__ wxprev, const uint32_t *__restrict__ waprev, float *__restrict__ f,
    int32_t *__restrict__ win_x, uint32_t *__restrict__ win_a) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= n) return;
    const uint64_t kv = key[j];
    const float sd = seed[j];
    if (d > 0 && kv == 0) {
        // the value comes from a facet: inherit its winner
        if (lane == 0) {
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
            int fa[4] = {(int)(pa & 255), (int)((pa >> 8) & 255), (int)((pa >> 16) & 255), (int)(pa >> 24)};
            int aa[4] = {0, 0, 0, 0};
            for (int i = 0, src = 0; i <= d; ++i) aa[i] = (i == fi) ? 0 : fa[src++];
            f[j] = sd;
            win_x[j] = wxprev[fac[fi]];
            win_a[j] = pack_comp(aa);
        }
        return;
    }
    // the simplex's own sample wins (vertices always search their own point)
    int lo_b = 0, hi_b = B;
    while (hi_b - lo_b > 1) {
        int mid = (lo_b + hi_b) >> 1;
        if (s_off[mid] <= j) lo_b = mid;
        else hi_b = mid;
    }
    const GridParam g = gp[lo_b];
    int comp[4] = {0, 0, 0, 0};
    float v = 0.f;
    if (d == 0) {
        comp[0] = k;
        v = kv ? key_value(kv) : 0.f;
    } else {
        unrank_interior((int)(0xffffffffu - (uint32_t)(kv & 0xffffffffu)), d, k, comp);
        v = key_value(kv);
    }
    int32_t vv[4];
    simplex_vertices(simp, d, j, vv);
    float sx, sy, sz;
    sample_point(L, vv, comp, d, k, sx, sy, sz);
    const float r = v * (1.0f + 1e-6f) + g.eps + 1e-30f;
    const int x0 = cell_of(sx - r, g.ox, g.inv_h, g.nx), x1 = cell_of(sx + r, g.ox, g.inv_h, g.nx);
    const int y0 = cell_of(sy - r, g.oy, g.inv_h, g.ny), y1 = cell_of(sy + r, g.oy, g.inv_h, g.ny);
    const int z0 = cell_of(sz - r, g.oz, g.inv_h, g.nz), z1 = cell_of(sz + r, g.oz, g.inv_h, g.nz);
    const int ny_ = y1 - y0 + 1;
    const int nrow = ny_ * (z1 - z0 + 1);
    float bd = INFINITY;
    int32_t bi = 0x7fffffff;
    for (int rr = lane; rr < nrow; rr += 64) {
        const int z = z0 + rr / ny_, y = y0 + rr % ny_;
        const int64_t c0 = g.cell_base + ((int64_t)z * g.ny + y) * g.nx + x0;
        const uint32_t p0 = cs[c0], p1 = cs[c0 + (x1 - x0) + 1];
        for (uint32_t p = p0; p < p1; ++p) {
            const float4 q = xs[p];
            const float dd = dist2(sx, sy, sz, q.x, q.y, q.z);
            const int32_t qi = __float_as_int(q.w);
            if (dd < bd || (dd == bd && qi < bi)) {
                bd = dd;
                bi = qi;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float od = __shfl_xor(bd, o, 64);
        const int32_t oi = __shfl_xor(bi, o, 64);
        if (od < bd || (od == bd && oi < bi)) {
            bd = od;
            bi = oi;
        }
    }
    if (lane == 0) {
        f[j] = d == 0 ? __fsqrt_rn(bd) : v;
        win_x[j] = bi;
        win_a[j] = pack_comp(comp);
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
    bytes += sizeof(float) * (nmax + 1) + 256;        // seed
    bytes += sizeof(uint64_t) * (nmax + 1) + 256;     // key
    bytes += 4 * (sizeof(int64_t) * (pb->B + 1) + 256); // tile offsets
    bytes += 1024;
    if (sz) {
        for (int d = 0; d < 4; ++d) sz->n[d] = n[d];
        sz->total_pts = pb->x_off[pb->B];
        sz->total_cells = tc;
    }
    return bytes;
}

template <int T>
static void launch_tiles(const TileArgs &ta, int wpb, hipStream_t s, const float *L, const int32_t *lxidx,
                         const int32_t *simp, const int64_t *s_off, const int64_t *tile_off, const float *seed,
                         uint64_t *key, const GridWork &g, uint64_t *evals) {
    const int64_t nb = (ta.n_tiles + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_flood_tiles<T>, dim3((unsigned)nb), dim3(64 * wpb), 0, s, ta, L, lxidx, simp, s_off, tile_off,
                       seed, key, g.gp, g.cell_start, g.xs, (unsigned long long *)evals);
}

hipError_t flood_run(const flood_problem *pb, const flood_tuning &tu, const flood_outputs *out, void *ws,
                     size_t ws_bytes, hipStream_t s) {
    FloodSizes sz;
    flood_workspace(pb, tu.cells_per_point, &sz);
    Carve c(ws, ws_bytes);
    GridWork g;
    grid_carve(c, pb->B, sz.total_pts, sz.total_cells, g);
    int64_t nmax = 0;
    for (int d = 0; d < 4; ++d) nmax = sz.n[d] > nmax ? sz.n[d] : nmax;
    float *seed = c.take<float>(nmax + 1);
    uint64_t *key = c.take<uint64_t>(nmax + 1);
    int64_t *tile_off[4];
    for (int d = 0; d < 4; ++d) tile_off[d] = c.take<int64_t>(pb->B + 1);
    if (!c.ok()) return hipErrorOutOfMemory;

    hipError_t e = grid_build(pb->X, pb->B, pb->x_off, pb->x_off_d, tu.cells_per_point, g, s);
    if (e != hipSuccess) return e;
    const int T = tu.samples_per_lane;
    const int wpb = tu.waves_per_block;
    for (int d = 0; d < 4; ++d) {
        const int64_t n = sz.n[d];
        if (n == 0) continue;
        const int64_t nint = n_interior(d, pb->k);
        const int64_t *soff_h = d == 0 ? pb->l_off : pb->s_off[d];
        const int64_t *soff_d = d == 0 ? pb->l_off_d : pb->s_off_d[d];
        const int32_t *simp = d == 0 ? nullptr : pb->simp[d];
        hipLaunchKernelGGL(k_seed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, n, pb->simp[1],
                           pb->tri_edges, pb->tet_tris, d > 0 ? out->f[d - 1] : nullptr, seed);
        e = fill_u64(key, 0ull, n, s);
        if (e != hipSuccess) return e;
        if (nint > 0) {
            const int64_t tsamp = 64 * (int64_t)T;
            int64_t ntiles = 0;
            for (int32_t b = 0; b < pb->B; ++b) ntiles += ((soff_h[b + 1] - soff_h[b]) * nint + tsamp - 1) / tsamp;
            hipLaunchKernelGGL(k_tile_off, dim3(1), dim3(1), 0, s, soff_d, pb->B, nint, tsamp, tile_off[d]);
            if (ntiles > 0) {
                TileArgs ta;
                ta.d = d;
                ta.k = pb->k;
                ta.n_int = (int32_t)nint;
                ta.landmarks_in_x = pb->landmarks_in_x;
                ta.B = pb->B;
                ta.pad = 0;
                ta.n_tiles = ntiles;
                if (out->tile_events[2 * d]) {
                    e = hipEventRecord((hipEvent_t)out->tile_events[2 * d], s);
                    if (e != hipSuccess) return e;
                }
                if (T == 1) launch_tiles<1>(ta, wpb, s, pb->Lxyz, pb->l_xidx, simp, soff_d, tile_off[d], seed, key, g, out->evals);
                else if (T == 2) launch_tiles<2>(ta, wpb, s, pb->Lxyz, pb->l_xidx, simp, soff_d, tile_off[d], seed, key, g, out->evals);
                else launch_tiles<4>(ta, wpb, s, pb->Lxyz, pb->l_xidx, simp, soff_d, tile_off[d], seed, key, g, out->evals);
                if (out->tile_events[2 * d + 1]) {
                    e = hipEventRecord((hipEvent_t)out->tile_events[2 * d + 1], s);
                    if (e != hipSuccess) return e;
                }
            }
        }
        const int64_t wblocks = (n + 3) / 4;
        hipLaunchKernelGGL(k_winner, dim3((unsigned)wblocks), dim3(256), 0, s, d, pb->k, n, pb->Lxyz, simp,
                           pb->tri_edges, pb->tet_tris, soff_d, pb->B, seed, key, g.gp, g.cell_start, g.xs,
                           d > 0 ? out->f[d - 1] : nullptr, d > 0 ? out->win_x[d - 1] : nullptr,
                           d > 0 ? out->win_a[d - 1] : nullptr, out->f[d], out->win_x[d], out->win_a[d]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace flood
