// C ABI of libflood: argument validation (before any launch), workspace
// queries and error reporting.  Kernels live in the .hip files.
#include <cmath>
#include <mutex>
#include <string>

#include "sample.hpp"

namespace flood_host {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace flood_host

using flood_host::set_error;

extern "C" const char *flood_last_error(void) { return flood_host::g_err.c_str(); }

namespace {

flood_status fail(flood_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

flood_status hip_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return FLOOD_OK;
    if (e == hipErrorOutOfMemory) return fail(FLOOD_ENOMEM, std::string(where) + ": workspace too small");
    return fail(FLOOD_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool offsets_ok(const int64_t *off, int32_t B) {
    if (!off || off[0] != 0) return false;
    for (int32_t b = 0; b < B; ++b)
        if (off[b + 1] < off[b]) return false;
    return true;
}

constexpr int64_t kMaxPoints = (int64_t)1 << 31;  // point rows travel as int32 / float bits

flood_tuning default_tuning(const flood_tuning *t) {
    flood_tuning r;
    r.cells_per_point = 1.0f;
    r.samples_per_lane = 1;
    r.waves_per_block = 4;
    r.tile_shells = 6;
    r.tile_extent = 24;
    r.queue_grab = 0;
    r.tile_lanes = 0;
    if (t) {
        if (t->cells_per_point != 0) r.cells_per_point = t->cells_per_point;
        if (t->samples_per_lane != 0) r.samples_per_lane = t->samples_per_lane;
        if (t->waves_per_block != 0) r.waves_per_block = t->waves_per_block;
        if (t->tile_shells != 0) r.tile_shells = t->tile_shells;
        if (t->tile_extent != 0) r.tile_extent = t->tile_extent;
        r.queue_grab = t->queue_grab;
        r.tile_lanes = t->tile_lanes;
    }
    return r;
}

flood_status check_tuning(const flood_tuning &t) {
    if (!(t.cells_per_point >= 0.05f && t.cells_per_point <= 64.f))
        return fail(FLOOD_EINVAL, "tuning: cells_per_point outside [0.05, 64]");
    if (t.samples_per_lane != 1 && t.samples_per_lane != 2 && t.samples_per_lane != 4)
        return fail(FLOOD_EINVAL, "tuning: samples_per_lane must be 1, 2 or 4");
    if (t.waves_per_block < 1 || t.waves_per_block > 4) return fail(FLOOD_EINVAL, "tuning: waves_per_block outside [1, 4]");
    if (t.tile_shells < -1 || t.tile_shells > 32 || t.tile_shells == 0)
        return fail(FLOOD_EINVAL, "tuning: tile_shells must be -1 or in [1, 32]");
    if (t.tile_extent < 2 || t.tile_extent > 64) return fail(FLOOD_EINVAL, "tuning: tile_extent outside [2, 64]");
    if (t.queue_grab != 0 && t.queue_grab != 1 && t.queue_grab != 2 && t.queue_grab != 4 && t.queue_grab != 8)
        return fail(FLOOD_EINVAL, "tuning: queue_grab must be 0, 1, 2, 4 or 8");
    if (t.tile_lanes != 0 && t.tile_lanes != 16 && t.tile_lanes != 32 && t.tile_lanes != 64)
        return fail(FLOOD_EINVAL, "tuning: tile_lanes must be 0, 16, 32 or 64");
    return FLOOD_OK;
}

flood_status check_problem(const flood_problem *pb) {
    if (!pb) return fail(FLOOD_EINVAL, "problem is NULL");
    if (pb->B < 1) return fail(FLOOD_EINVAL, "problem: B must be >= 1");
    if (pb->k < 1) return fail(FLOOD_EINVAL, "problem: k must be >= 1");
    if (pb->sampling != FLOOD_SAMPLING_GRID && pb->sampling != FLOOD_SAMPLING_RANDOM)
        return fail(FLOOD_EINVAL, "problem: sampling must be FLOOD_SAMPLING_GRID or FLOOD_SAMPLING_RANDOM");
    if (pb->sampling == FLOOD_SAMPLING_GRID && pb->k > 255)
        return fail(FLOOD_EUNSUPPORTED, "problem: k > 255 (compositions are packed in 8 bits)");
    if (pb->sampling == FLOOD_SAMPLING_RANDOM && pb->k > 65536)
        return fail(FLOOD_EUNSUPPORTED, "problem: more than 65536 random samples per simplex");
    if (pb->landmarks_in_x != 0 && pb->landmarks_in_x != 1) return fail(FLOOD_EINVAL, "problem: landmarks_in_x must be 0 or 1");
    if (!pb->X || !pb->x_off_d || !pb->Lxyz || !pb->l_off_d) return fail(FLOOD_EINVAL, "problem: NULL device pointer");
    if (pb->landmarks_in_x && !pb->l_xidx) return fail(FLOOD_EINVAL, "problem: landmarks_in_x needs l_xidx");
    if (!offsets_ok(pb->x_off, pb->B)) return fail(FLOOD_EINVAL, "problem: x_off must start at 0 and be non-decreasing");
    if (!offsets_ok(pb->l_off, pb->B)) return fail(FLOOD_EINVAL, "problem: l_off must start at 0 and be non-decreasing");
    if (pb->x_off[pb->B] >= kMaxPoints) return fail(FLOOD_EUNSUPPORTED, "problem: more than 2^31 - 1 points");
    for (int d = 1; d < 4; ++d) {
        if (!offsets_ok(pb->s_off[d], pb->B)) return fail(FLOOD_EINVAL, "problem: s_off must start at 0 and be non-decreasing");
        if (pb->s_off[d][pb->B] > 0 && (!pb->simp[d] || !pb->s_off_d[d]))
            return fail(FLOOD_EINVAL, "problem: NULL simplex array");
        if (pb->s_off[d][pb->B] >= kMaxPoints) return fail(FLOOD_EUNSUPPORTED, "problem: too many simplices");
    }
    for (int d = 0; d < 4; ++d) {
        const int64_t *so = d == 0 ? pb->l_off : pb->s_off[d];
        const int64_t nint = flood::own_samples(d, pb->k, pb->sampling);
        if (so[pb->B] * nint >= ((int64_t)1 << 31))
            return fail(FLOOD_EUNSUPPORTED, "problem: more than 2^31 - 1 interior samples in one dimension");
        int64_t bk = 0;
        for (int32_t b = 0; b < pb->B; ++b) bk += (int64_t)1 << (3 * flood::morton_bits((so[b + 1] - so[b]) * nint));
        if (bk >= ((int64_t)1 << 32) - 1) return fail(FLOOD_EUNSUPPORTED, "problem: too many clouds for the sample sort");
    }
    if (pb->s_off[2][pb->B] > 0 && !pb->tri_edges) return fail(FLOOD_EINVAL, "problem: tri_edges is NULL");
    if (pb->s_off[3][pb->B] > 0 && !pb->tet_tris) return fail(FLOOD_EINVAL, "problem: tet_tris is NULL");
    for (int32_t b = 0; b < pb->B; ++b) {
        int64_t nsimp = pb->l_off[b + 1] - pb->l_off[b];
        if (nsimp > 0 && pb->x_off[b + 1] == pb->x_off[b])
            return fail(FLOOD_EINVAL, "problem: a cloud with landmarks has no points");
    }
    return FLOOD_OK;
}

flood_status check_outputs(const flood_problem *pb, const flood_outputs *out, const char *name) {
    if (!out) return fail(FLOOD_EINVAL, std::string(name) + ": outputs are NULL");
    int with_w = 0, dims = 0;
    for (int d = 0; d < 4; ++d) {
        int64_t n = d == 0 ? pb->l_off[pb->B] : pb->s_off[d][pb->B];
        if (n > 0 && (!out->f[d] || !out->win_x[d] || !out->win_a[d]))
            return fail(FLOOD_EINVAL, std::string(name) + ": NULL output array");
        if (n > 0) {
            ++dims;
            with_w += out->win_w[d] != nullptr;
        }
    }
    if (with_w != 0 && with_w != dims)
        return fail(FLOOD_EINVAL, std::string(name) + ": win_w must be given for every dimension or for none");
    return FLOOD_OK;
}

}  // namespace

extern "C" size_t flood_fps_workspace_size(int32_t B, const int64_t *x_off, const int32_t *n_lm) {
    if (B < 1 || !offsets_ok(x_off, B) || !n_lm) return 0;
    return flood::fps_workspace(B, x_off, n_lm);
}

extern "C" flood_status flood_fps(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                                  const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d, int32_t *idx,
                                  float *radius, void *ws, size_t ws_bytes, void *stream) {
    if (!X || !x_off_d || !n_lm || !n_lm_d || !idx) return fail(FLOOD_EINVAL, "flood_fps: NULL pointer");
    if (B < 1) return fail(FLOOD_EINVAL, "flood_fps: B must be >= 1");
    if (!offsets_ok(x_off, B)) return fail(FLOOD_EINVAL, "flood_fps: x_off must start at 0 and be non-decreasing");
    if (x_off[B] >= kMaxPoints) return fail(FLOOD_EUNSUPPORTED, "flood_fps: more than 2^31 - 1 points");
    for (int32_t b = 0; b < B; ++b)
        if (n_lm[b] < 1 || n_lm[b] > x_off[b + 1] - x_off[b])
            return fail(FLOOD_EINVAL, "flood_fps: need 1 <= n_lm[b] <= N_b");
    size_t need = flood::fps_workspace(B, x_off, n_lm);
    if (!ws || ws_bytes < need) return fail(FLOOD_ENOMEM, "flood_fps: workspace smaller than flood_fps_workspace_size");
    hipError_t e = flood::fps_run(X, B, x_off, x_off_d, n_lm, n_lm_d, start_d, idx, radius, ws, ws_bytes,
                                  (hipStream_t)stream);
    return hip_status(e, "flood_fps");
}

extern "C" size_t flood_filtration_workspace_size(const flood_problem *pb, const flood_tuning *tune) {
    if (check_problem(pb) != FLOOD_OK) return 0;
    flood_tuning t = default_tuning(tune);
    if (check_tuning(t) != FLOOD_OK) return 0;
    return flood::flood_workspace(pb, t.cells_per_point, nullptr);
}

extern "C" flood_status flood_filtration(const flood_problem *pb, const flood_tuning *tune, const flood_outputs *out,
                                         void *ws, size_t ws_bytes, void *stream) {
    flood_status st = check_problem(pb);
    if (st != FLOOD_OK) return st;
    flood_tuning t = default_tuning(tune);
    st = check_tuning(t);
    if (st != FLOOD_OK) return st;
    st = check_outputs(pb, out, "flood_filtration");
    if (st != FLOOD_OK) return st;
    size_t need = flood::flood_workspace(pb, t.cells_per_point, nullptr);
    if (!ws || ws_bytes < need)
        return fail(FLOOD_ENOMEM, "flood_filtration: workspace smaller than flood_filtration_workspace_size");
    hipError_t e = flood::flood_run(pb, t, out, ws, ws_bytes, (hipStream_t)stream);
    return hip_status(e, "flood_filtration");
}

extern "C" flood_status flood_filtration_backward(const flood_problem *pb, const flood_outputs *fwd,
                                                  const float *const grad_f[4], float *grad_X, float *grad_L,
                                                  void *stream) {
    flood_status st = check_problem(pb);
    if (st != FLOOD_OK) return st;
    if (!fwd || !grad_f) return fail(FLOOD_EINVAL, "flood_filtration_backward: NULL argument");
    for (int d = 0; d < 4; ++d) {
        int64_t n = d == 0 ? pb->l_off[pb->B] : pb->s_off[d][pb->B];
        if (n > 0 && grad_f[d] && (!fwd->win_x[d] || !fwd->win_a[d]))
            return fail(FLOOD_EINVAL, "flood_filtration_backward: NULL winner array");
        if (n > 0 && grad_f[d] && pb->sampling == FLOOD_SAMPLING_RANDOM && !fwd->win_w[d])
            return fail(FLOOD_EINVAL, "flood_filtration_backward: random sample sets need the winners' weights (win_w)");
    }
    hipError_t e = flood::backward_run(pb, fwd, grad_f, grad_X, grad_L, (hipStream_t)stream);
    return hip_status(e, "flood_filtration_backward");
}

// ---------------------------------------------------------------------------
// allocation-free filtration: the workspace is one static device array per
// device, located once per device with hipGetSymbolAddress (in host code the
// array's name is not a device address; only the looked-up pointer is used)

static __device__ __align__(256) unsigned char scratch[FLOOD_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// the current device's scratch address, looked up on the first call there
hipError_t scratch_ptr(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" flood_status flood_filtration_noalloc(const flood_problem *pb, const flood_tuning *tune,
                                                 const flood_outputs *out, void *stream) {
    flood_status st = check_problem(pb);
    if (st != FLOOD_OK) return st;
    flood_tuning t = default_tuning(tune);
    st = check_tuning(t);
    if (st != FLOOD_OK) return st;
    st = check_outputs(pb, out, "flood_filtration_noalloc");
    if (st != FLOOD_OK) return st;
    const size_t need = flood::flood_workspace(pb, t.cells_per_point, nullptr);
    if (need > FLOOD_STATIC_SCRATCH_BYTES)
        return fail(FLOOD_ENOMEM, "flood_filtration_noalloc: the problem needs " + std::to_string(need) +
                                      " bytes of workspace, more than the static scratch of " +
                                      std::to_string((size_t)FLOOD_STATIC_SCRATCH_BYTES) +
                                      " bytes; use flood_filtration with a caller workspace");
    void *ws = nullptr;
    hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) return hip_status(e, "flood_filtration_noalloc: scratch lookup");
    e = flood::flood_run(pb, t, out, ws, FLOOD_STATIC_SCRATCH_BYTES, (hipStream_t)stream);
    return hip_status(e, "flood_filtration_noalloc");
}
