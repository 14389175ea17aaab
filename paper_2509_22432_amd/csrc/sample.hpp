// Device helpers shared by the forward, winner and backward kernels: the
// barycentric sample grid of Lemma 6 (P = {sum_i (a_i/k) v_i}), its interior
// enumeration, and the direct-difference squared distance.
#pragma once
#include "internal.hpp"

namespace flood {

// Morton resolution (bits per axis) of the sample sort: about four samples
// per bucket on a 2^m cube
__host__ __device__ inline int morton_bits(int64_t S) {
    int m = 1;
    while (m < 8 && ((int64_t)4 << (3 * m)) < S) ++m;
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

// sample point s = sum_i (a_i/k) v_i in float32 (shared by forward, winner
// search and backward so all three see the same coordinates)
__device__ __forceinline__ void sample_point(const float *__restrict__ L, const int32_t *v, const int *a, int d, int k,
                                             float &sx, float &sy, float &sz) {
    // w = a_i/k correctly rounded: w = 1 exactly for a vertex sample and
    // w = 0 terms add nothing, so a vertex sample is the vertex itself
    sx = 0.f;
    sy = 0.f;
    sz = 0.f;
    for (int i = 0; i <= d; ++i) {
        const float w = __fdiv_rn((float)a[i], (float)k);
        sx = __fmaf_rn(w, L[3 * v[i]], sx);
        sy = __fmaf_rn(w, L[3 * v[i] + 1], sy);
        sz = __fmaf_rn(w, L[3 * v[i] + 2], sz);
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
