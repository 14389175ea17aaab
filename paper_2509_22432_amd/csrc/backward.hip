// Backward of the flood values.  Away from ties, f(sigma) = ||s* - x*|| with
// s* = sum_i w_i v_i the winning sample (grid sets: w_i = a_i/k; random
// sets: the recorded weights) and x* its nearest point, so the derivative
// routes -g u to x* and g w_i u to each vertex v_i, with
// u = (s* - x*) / ||s* - x*|| (u = 0 when f = 0).  One thread per simplex;
// float atomics accumulate into the caller's gradients.
#include "sample.hpp"

namespace flood {

__global__ void k_backward(int d, int k, int64_t n, int64_t n_pts, const float *__restrict__ X, const float *__restrict__ L,
                           const int32_t *__restrict__ simp, const float *__restrict__ gf,
                           const int32_t *__restrict__ win_x, const uint32_t *__restrict__ win_a,
                           const float *__restrict__ win_w, float *__restrict__ gX, float *__restrict__ gL) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float g = gf[j];
    if (g == 0.f) return;
    float w[4];
    if (win_w) {
        const float4 ww = *(const float4 *)&win_w[4 * j];
        w[0] = ww.x; w[1] = ww.y; w[2] = ww.z; w[3] = ww.w;
    } else {
        const uint32_t pa = win_a[j];
        const int a[4] = {(int)(pa & 255), (int)((pa >> 8) & 255), (int)((pa >> 16) & 255), (int)(pa >> 24)};
        grid_weights(a, d, k, w);
    }
    int32_t v[4];
    simplex_vertices(simp, d, j, v);
    float sx, sy, sz;
    weighted_point(L, v, w, d, sx, sy, sz);
    const int64_t xi = win_x[j];
    if (xi < 0 || xi >= n_pts) return;  // no winner point recorded: no gradient
    const float dx = sx - X[3 * xi], dy = sy - X[3 * xi + 1], dz = sz - X[3 * xi + 2];
    const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
    if (!(nrm > 0.f)) return;
    const float s = g / nrm;
    const float ux = dx * s, uy = dy * s, uz = dz * s;
    if (gX) {
        atomicAdd(&gX[3 * xi], -ux);
        atomicAdd(&gX[3 * xi + 1], -uy);
        atomicAdd(&gX[3 * xi + 2], -uz);
    }
    if (gL) {
        for (int i = 0; i <= d; ++i) {
            if (w[i] == 0.f) continue;
            atomicAdd(&gL[3 * v[i]], w[i] * ux);
            atomicAdd(&gL[3 * v[i] + 1], w[i] * uy);
            atomicAdd(&gL[3 * v[i] + 2], w[i] * uz);
        }
    }
}

hipError_t backward_run(const flood_problem *pb, const flood_outputs *fwd, const float *const grad_f[4],
                        float *grad_X, float *grad_L, hipStream_t s) {
    for (int d = 0; d < 4; ++d) {
        const int64_t n = d == 0 ? pb->l_off[pb->B] : pb->s_off[d][pb->B];
        if (n == 0 || grad_f[d] == nullptr) continue;
        hipLaunchKernelGGL(k_backward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, pb->k, n, pb->x_off[pb->B], pb->X,
                           pb->Lxyz, d == 0 ? nullptr : pb->simp[d], grad_f[d], fwd->win_x[d], fwd->win_a[d],
                           pb->sampling == FLOOD_SAMPLING_RANDOM ? fwd->win_w[d] : nullptr, grad_X, grad_L);
    }
    return hipGetLastError();
}

}  // namespace flood
