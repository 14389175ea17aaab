// Device helpers shared by the forward, winner and backward kernels: the
// barycentric sample grid of Lemma 6 (P = {sum_i (a_i/k) v_i}), its interior
// enumeration, and the direct-difference squared distance.
#pragma once
#include "internal.hpp"

namespace flood {

// Morton resolution (bits per axis) of the sample sort: 2 to 16 samples per
// bucket of a 2^m cube on average (a tile spans a few buckets; neighbouring
// samples share a bucket, so the counting pass takes one atomic per bucket
// and wavefront)
__host__ __device__ inline int morton_bits(int64_t S) {
    int m = 1;
    while (m < 8 && ((int64_t)16 << (3 * m)) < S) ++m;
    return m;
}

// correctly rounded float square root.  The rounded-sqrt intrinsic of the
// HIP headers lowers to the approximate hardware instruction unless the
// rounded-operation macros are defined, which made flood values depend on
// the kernel that published them; the builtin is lowered with the exact
// correction steps.
__device__ __forceinline__ float sqrt_rn(float x) { return __builtin_sqrtf(x); }

__device__ __forceinline__ float dist2(float sx, float sy, float sz, float px, float py, float pz) {
    const float dx = sx - px, dy = sy - py, dz = sz - pz;
    return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
}

// number of compositions of n into p >= 1 non-negative parts, p <= 3
__device__ __forceinline__ int ncomp(int n, int p) {
    return p == 1 ? 1 : (p == 2 ? n + 1 : (n + 1) * (n + 2) / 2);
}

// q-th interior composition (all parts >= 1) of k into d+1 parts, in
// lexicographically descending order; a[0..d]
__device__ __forceinline__ void unrank_interior(int q, int d, int k, int a[4]) {
    int rem = k - (d + 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = 0;
    for (int i = 0; i < d; ++i) {
        int v = rem;
        for (; v > 0; --v) {
            int c = ncomp(rem - v, d - i);
            if (q < c) break;
            q -= c;
        }
        a[i] = v + 1;
        rem -= v;
    }
    a[d] = rem + 1;
}

__host__ __device__ inline int64_t n_interior(int d, int k) {
    if (d == 0) return 1;
    int64_t m = k - 1;  // C(k-1, d)
    if (m < d) return 0;
    if (d == 1) return m;
    if (d == 2) return m * (m - 1) / 2;
    return m * (m - 1) * (m - 2) / 6;
}

// s = sum_i w_i v_i in float32, one fused multiply-add per term in vertex
// order (shared by forward, winner search and backward so all three see the
// same coordinates; w = 0 terms add nothing, so a face's sample keeps its
// bits when it is written over the coface's vertices)
__device__ __forceinline__ void weighted_point(const float *__restrict__ L, const int32_t *v, const float *w, int d,
                                               float &sx, float &sy, float &sz) {
    sx = 0.f;
    sy = 0.f;
    sz = 0.f;
    for (int i = 0; i <= d; ++i) {
        sx = __fmaf_rn(w[i], L[3 * v[i]], sx);
        sy = __fmaf_rn(w[i], L[3 * v[i] + 1], sy);
        sz = __fmaf_rn(w[i], L[3 * v[i] + 2], sz);
    }
}

// grid weights w_i = a_i / k, correctly rounded (w = 1 exactly for a vertex
// sample, so a vertex sample is the vertex itself)
__device__ __forceinline__ void grid_weights(const int *a, int d, int k, float w[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = i <= d ? __fdiv_rn((float)a[i], (float)k) : 0.f;
}

// sample point s = sum_i (a_i/k) v_i of the barycentric grid (Lemma 6)
__device__ __forceinline__ void sample_point(const float *__restrict__ L, const int32_t *v, const int *a, int d, int k,
                                             float &sx, float &sy, float &sz) {
    float w[4];
    grid_weights(a, d, k, w);
    weighted_point(L, v, w, d, sx, sy, sz);
}

// ---------------------------------------------------------------------------
// random sample sets (Thm. 5 holds for any finite P_sigma inside conv sigma;
// Lemma 9 draws the points uniformly).  Draws come from the counter-based
// generator Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011), written
// from its published definition: sample q of the simplex in cloud-local row
// r of dimension d uses counter (q, r, d, 0) and key (seed, 0); the top 24
// bits of words 0..d-1 give uniforms u_i = (word >> 40) 2^-24 (exact in
// float32), and the spacings of the sorted u_(1) <= .. <= u_(d),
// (u_(1), u_(2) - u_(1), .., 1 - u_(d)), are uniform on the simplex
// (Dirichlet(1, .., 1)); every spacing is a multiple of 2^-24 and exact.

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t mul0 = 0xD2E7470EE14C6C93ull, mul1 = 0xCA5A826395121157ull;  // round multipliers
    const uint64_t weyl0 = 0x9E3779B97F4A7C15ull, weyl1 = 0xBB67AE8584CAA73Bull;  // key schedule
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(mul0, c[0]), lo0 = mul0 * c[0];
        const uint64_t hi1 = __umul64hi(mul1, c[2]), lo1 = mul1 * c[2];
        const uint64_t x0 = hi1 ^ c[1] ^ k0, x2 = hi0 ^ c[3] ^ k1;
        c[0] = x0;
        c[1] = lo1;
        c[2] = x2;
        c[3] = lo0;
        k0 += weyl0;
        k1 += weyl1;
    }
}

__device__ __forceinline__ void random_weights(int d, uint32_t q, int64_t row, uint64_t seed, float w[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = 0.f;
    if (d == 0) {
        w[0] = 1.f;
        return;
    }
    uint64_t c[4] = {(uint64_t)q, (uint64_t)row, (uint64_t)d, 0ull};
    philox4x64_10(c, seed, 0ull);
    float u[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) u[i] = (float)(uint32_t)(c[i] >> 40) * 0x1p-24f;
    // sort the first d uniforms (d <= 3): a three-element network
    if (d >= 2 && u[1] < u[0]) { const float t = u[0]; u[0] = u[1]; u[1] = t; }
    if (d == 3) {
        if (u[2] < u[1]) { const float t = u[1]; u[1] = u[2]; u[2] = t; }
        if (u[1] < u[0]) { const float t = u[0]; u[0] = u[1]; u[1] = t; }
    }
    w[0] = u[0];
    for (int i = 1; i < d; ++i) w[i] = u[i] - u[i - 1];
    w[d] = 1.f - u[d - 1];
}

// how a simplex's own samples are drawn
struct SampleRule {
    int32_t k;         // grid: segments per edge; random: samples per simplex
    int32_t sampling;  // FLOOD_SAMPLING_GRID or FLOOD_SAMPLING_RANDOM
    uint64_t seed;     // random sets only
};

// own samples of a d-simplex: the interior grid points (all a_i >= 1; the
// boundary points belong to the faces) or the m random points; a vertex owns
// itself
__host__ __device__ inline int64_t own_samples(int d, int k, int sampling) {
    if (d == 0) return 1;
    return sampling == FLOOD_SAMPLING_RANDOM ? (int64_t)k : n_interior(d, k);
}

// weights of own sample q of the simplex in cloud-local row `row`
__device__ __forceinline__ void own_weights(const SampleRule &r, int d, int q, int64_t row, float w[4]) {
    if (r.sampling == FLOOD_SAMPLING_RANDOM) {
        random_weights(d, (uint32_t)q, row, r.seed, w);
    } else {
        int comp[4];
        if (d == 0) {
            comp[0] = r.k;
            comp[1] = comp[2] = comp[3] = 0;
        } else {
            unrank_interior(q, d, r.k, comp);
        }
        grid_weights(comp, d, r.k, w);
    }
}

__device__ __forceinline__ void simplex_vertices(const int32_t *__restrict__ simp, int d, int64_t j, int32_t v[4]) {
    if (d == 0) {
        v[0] = (int32_t)j;
        return;
    }
    for (int i = 0; i <= d; ++i) v[i] = simp[j * (d + 1) + i];
}

__device__ __forceinline__ int cell_of(float v, float o, float inv_h, int n) {
    float t = (v - o) * inv_h;
    int c = (t >= 0.f) ? (int)fminf(t, (float)(n - 1)) : 0;
    return c;
}

// bijective block -> work remap so consecutive tiles share an XCD (and its L2)
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
    const int64_t q = nb / 8, r = nb % 8;
    const int64_t x = bid % 8, i = bid / 8;
    return x * q + (x < r ? x : r) + i;
}

}  // namespace flood
