/*
 * flood.h -- C ABI of the MI355X (gfx950) flooding library.
 *
 * The library computes the filtration of the Flood complex (Graf et al.,
 * "The Flood Complex", NeurIPS 2025): for every simplex sigma of the
 * Delaunay triangulation of a landmark set L, the sampled flood value
 *
 *     f(sigma) = max over faces tau of sigma, max over p in P_tau of
 *                min over x in X of ||p - x||                      (1)
 *
 * (Def. 1 with the sample sets of Sec. 4.1 "Approximation"), where P_tau is
 * the barycentric grid of Lemma 6 with k segments (k+1 points) per edge:
 * P_tau = { sum_i (a_i/k) v_i : a_i >= 0 integers, sum_i a_i = k }.
 *
 * Conventions for every entry point:
 *  - Plain C types only.  "device" pointers are HIP device memory on the
 *    current device, "host" pointers are ordinary host memory.
 *  - Every call returns a flood_status; nothing throws or aborts.  On a
 *    non-OK status flood_last_error() returns a thread-local message.
 *  - All argument validation happens before any kernel is launched; a
 *    rejected call launches nothing and writes nothing.
 *  - Device-side calls are asynchronous on `stream` (a hipStream_t; NULL is
 *    the default stream).  A launch failure is returned as FLOOD_EHIP; a
 *    fault inside a kernel surfaces at the caller's next synchronisation.
 *  - The library allocates no device memory: callers pass a workspace of at
 *    least the size returned by the matching *_workspace_size query (any
 *    alignment; the library aligns internally).  This keeps every device
 *    entry point capturable in a HIP graph.  Calls that share a workspace
 *    must not overlap.
 *  - Coordinates are float32, row-major [n][3], contiguous.
 */
#ifndef FLOOD_H
#define FLOOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t flood_status;
#define FLOOD_OK 0
#define FLOOD_EINVAL 1       /* bad argument (null pointer, size, NaN/Inf input, bad offsets) */
#define FLOOD_ENOMEM 2       /* workspace too small, or a host allocation failed */
#define FLOOD_EHIP 3         /* a HIP runtime call or kernel launch failed */
#define FLOOD_EDEGENERATE 4  /* degenerate geometry (see the entry point) */
#define FLOOD_EUNSUPPORTED 5 /* outside the supported range (e.g. k > 255) */

/* Message for the last non-OK status on this thread ("" if none). */
const char *flood_last_error(void);

/* ---------------------------------------------------------------------------
 * Farthest-point landmarks (Sec. 3.2: greedy k-centre,
 * a 2-approximation of the optimal covering radius; the paper's pipeline
 * selects landmarks this way, Sec. 5 and Table 1 "Landmark select.").
 *
 * B clouds are processed together.  Cloud b owns points
 * X[x_off[b] .. x_off[b+1]) and receives n_lm[b] landmarks in
 * idx[l_off[b] .. l_off[b]+n_lm[b]), where l_off is the exclusive prefix sum
 * of n_lm.  Indices are local to the cloud (0-based within it).
 *
 * Rule (bit-exact, float32): mind_i starts at +inf; for t = 0,1,..: with
 * landmark l_t, mind_i = min(mind_i, d2(x_i, l_t)) where
 * d2 = (dx*dx + dy*dy) + dz*dz, dx = x - l, every operation rounded to
 * float32, no fused multiply-add; l_{t+1} = argmax_i mind_i, lowest index
 * on ties; l_0 = start[b].  radius[l_off[b]+t] = sqrtf(max_i mind_i) after
 * landmarks 0..t, so the last entry is d_H(X_b, L_b).
 *
 *   X       device float [sum N][3]
 *   x_off   host int64 [B+1], x_off[0] = 0, non-decreasing
 *   x_off_d device int64 [B+1], same values
 *   n_lm    host int32 [B], 1 <= n_lm[b] <= N_b
 *   n_lm_d  device int32 [B], same values
 *   start_d device int64 [B] or NULL (all 0); must satisfy 0 <= start[b] < N_b
 *   idx     device int32 [sum n_lm]              (output)
 *   radius  device float [sum n_lm], or NULL     (output)
 * EDEGENERATE cannot be detected before the run: if a cloud has fewer
 * distinct points than landmarks, its remaining indices repeat an earlier
 * landmark and its radius reaches 0; callers check radius.
 * Clouds of at least 2^19 points (2^12 in calls of at most 8 clouds) run
 * as one cooperative launch each (one workgroup per CU exchanging candidates
 * through the workspace); the other clouds share one launch with a
 * workgroup per cloud.  The call
 * fails with FLOOD_EHIP if the device cannot co-schedule it.  Should the
 * workgroups stop hearing from each other (a poll limit of about 4M polls
 * per exchange), the launch ends and the cloud's undecided indices are -1:
 * callers that cannot rule that out check for negative indices.
 */
size_t flood_fps_workspace_size(int32_t B, const int64_t *x_off, const int32_t *n_lm);
flood_status flood_fps(const float *X, int32_t B, const int64_t *x_off, const int64_t *x_off_d,
                       const int32_t *n_lm, const int32_t *n_lm_d, const int64_t *start_d,
                       int32_t *idx, float *radius, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Delaunay triangulation of the landmarks, on the host (Sec. 4: Del(L) is
 * the simplex set; the paper uses CGAL/qhull).  Incremental insertion with
 * exactly evaluated orientation and in-sphere predicates (FP64 filter,
 * exact big-integer fallback), so the result is the exact Delaunay
 * triangulation of the given float32 coordinates.
 *
 *   Lxyz   host float [L][3], L >= 4, finite
 *   out    receives a library-owned handle; free it with flood_complex_free
 * EDEGENERATE: fewer than 4 affinely independent points, duplicate points,
 * or an exactly coplanar/cospherical configuration that decides the
 * triangulation (the paper assumes general position).
 */
typedef struct flood_complex flood_complex;
flood_status flood_delaunay(const float *Lxyz, int32_t L, flood_complex **out);
/* The same in ambient dimension 2 (Sec. 5.2 varies the ambient dimension):
 * Lxy host float [L][2], L >= 3; the complex has vertices, edges and
 * triangles only (no tetrahedra, tets / tet_tris export nothing), with
 * orientation and in-circle predicates evaluated exactly.  EDEGENERATE:
 * fewer than 3 non-collinear points, duplicates, or an exactly cocircular
 * configuration that decides the triangulation.  The flooding entry points
 * take such a complex with the points and landmarks as [n][3] rows whose
 * third coordinate is 0. */
flood_status flood_delaunay2d(const float *Lxy, int32_t L, flood_complex **out);
/* counts[0..3] = vertices, edges, triangles, tetrahedra; counts[4] = exact
 * predicate fallbacks taken (diagnostic). */
flood_status flood_complex_counts(const flood_complex *cx, int64_t counts[5]);
/* Copies the complex into caller-owned host arrays sized by the counts:
 * edges [E][2], tris [F][3], tets [T][4] -- each row sorted ascending, rows
 * in lexicographic order; tri_edges [F][3] and tet_tris [T][4] hold the
 * facet indices, facet i being the face without the row's i-th vertex.
 * Any output pointer may be NULL to skip it. */
flood_status flood_complex_export(const flood_complex *cx, int32_t *edges, int32_t *tris,
                                  int32_t *tets, int32_t *tri_edges, int32_t *tet_tris);
void flood_complex_free(flood_complex *cx);

/* ---------------------------------------------------------------------------
 * Persistence diagrams of a flood filtration over Z/2, dimensions 0..2, on
 * the host: the homology step that follows the flooding (the paper computes
 * it with Gudhi; Sec. 2 defines the sublevel filtration and the diagrams).
 * Simplices are ordered by (f, dimension, vertex tuple) and the boundary
 * matrix is reduced column by column with the clearing shortcut.
 *
 *   n[0..3]    simplices per dimension (vertices, edges, triangles, tets)
 *   edges      host int32 [n1][2] vertex rows; tri_edges [n2][3] and
 *              tet_tris [n3][4] facet rows, facet i omitting the row's
 *              i-th vertex -- exactly as flood_complex_export writes them.
 *              Rows of each dimension must be in lexicographic order of
 *              their sorted vertex tuples (ties in f are broken by it).
 *   f[d]       host float [n[d]] flood values with f(face) <= f(coface)
 *   out        receives a library-owned diagram; free with flood_diagram_free
 * EINVAL: NULL arguments, NaN, a face index out of range, or a face whose
 * value exceeds its coface's.  The diagram keeps pairs of positive
 * persistence and the essential classes (death = +inf).
 */
typedef struct flood_diagram flood_diagram;
flood_status flood_persistence(const int64_t n[4], const int32_t *edges, const int32_t *tri_edges,
                               const int32_t *tet_tris, const float *const f[4], flood_diagram **out);
/* counts[p] = points of the dimension-p diagram (finite pairs + essential). */
flood_status flood_diagram_counts(const flood_diagram *dg, int64_t counts[3]);
/* Copies the dimension-p points into caller-owned host arrays of
 * counts[p] entries: births, deaths (+inf for essential classes), and the
 * row of the birth simplex (dimension p) and of the death simplex
 * (dimension p+1; -1 if essential).  Finite pairs come in the filtration
 * order of their birth simplex, then the essential classes.  Any output
 * pointer may be NULL. */
flood_status flood_diagram_export(const flood_diagram *dg, int32_t dim, float *birth, float *death,
                                  int64_t *birth_row, int64_t *death_row);
void flood_diagram_free(flood_diagram *dg);

/* ---------------------------------------------------------------------------
 * Flood filtration (equation (1) above), B clouds at once.
 *
 * Cloud b owns points X[x_off[b]..x_off[b+1]), landmarks
 * Lxyz[l_off[b]..l_off[b+1]) and, for dimension d = 1,2,3, the simplices
 * simp[d][s_off[d][b]..s_off[d][b+1]).  Vertex ids inside simp[] are GLOBAL
 * landmark rows (already offset by l_off[b]); tri_edges / tet_tris hold
 * GLOBAL edge / triangle rows.  Rows of simp[d] must be sorted ascending
 * (the vertex order fixes the meaning of win_a).  The 0-simplices are the
 * landmarks themselves, in order.
 *
 * sampling selects the sample sets P_sigma:
 *  - FLOOD_SAMPLING_GRID (0): the barycentric grid of Lemma 6 with k
 *    segments per edge, k <= 255 (equation (1) above);
 *  - FLOOD_SAMPLING_RANDOM (1): every simplex of dimension >= 1 owns k
 *    points drawn uniformly from its convex hull (Thm. 5 holds for any
 *    finite P_sigma inside conv sigma; Lemma 9 bounds the covering radius of
 *    uniform draws), 1 <= k <= 65536, and f(sigma) = max(own value, max
 *    over facets f(tau)) -- the face sets are not subsets of the coface's
 *    here, so this closure of Sec. 4.1 is what makes f monotone.  Sample q
 *    of the simplex in cloud-local row r of dimension d is
 *    sum_i w_i v_i, the weights being the spacings of the sorted uniforms
 *    u_i = (word_i >> 40) * 2^-24, i < d, of Philox4x64-10 (Salmon et al.,
 *    SC 2011) at counter (q, r, d, 0) and key (seed, 0): u_(1),
 *    u_(2) - u_(1), ..., 1 - u_(d).  A vertex owns itself.
 *
 * landmarks_in_x = 1 supplies l_xidx, the global X row of each landmark
 * (for FPS landmarks, Lxyz[j] = X[l_xidx[j]]); it enables the per-sample
 * bound d(p, X) <= min_i ||p - X[l_xidx[v_i]]|| from the proof of Lemma 7,
 * which speeds the search and never changes a value.  The bound is taken
 * from X itself, so it holds even when Lxyz no longer equals those rows; a
 * row outside the landmark's own cloud contributes no bound.
 */
#define FLOOD_SAMPLING_GRID 0
#define FLOOD_SAMPLING_RANDOM 1
typedef struct {
    int32_t B;               /* number of clouds, >= 1 */
    int32_t k;               /* grid: segments per edge, 1..255 (k+1 samples per edge);
                                random: samples per simplex, 1..65536 */
    int32_t landmarks_in_x;  /* 0 or 1 (see above) */
    int32_t sampling;        /* FLOOD_SAMPLING_GRID or FLOOD_SAMPLING_RANDOM */
    const float *X;          /* device [sum N][3] */
    const int64_t *x_off;    /* host [B+1] */
    const int64_t *x_off_d;  /* device [B+1] */
    const float *Lxyz;       /* device [sum L][3] */
    const int32_t *l_xidx;   /* device [sum L]: global X row of each landmark (NULL if !landmarks_in_x) */
    const int64_t *l_off;    /* host [B+1] */
    const int64_t *l_off_d;  /* device [B+1] */
    const int32_t *simp[4];  /* device; simp[0] unused; simp[1] [E][2], simp[2] [F][3], simp[3] [T][4] */
    const int64_t *s_off[4]; /* host [B+1] per dimension (s_off[0] unused) */
    const int64_t *s_off_d[4]; /* device [B+1] per dimension (s_off_d[0] unused) */
    const int32_t *tri_edges; /* device [F][3] */
    const int32_t *tet_tris;  /* device [T][4] */
    uint64_t seed;            /* random sample sets: the generator's key */
} flood_problem;

/* Outputs, all device.  f[d] float [n_d]: the flood value (1).  win_x[d]
 * int32 [n_d]: global X row of the nearest point x* of the winning sample
 * s* (lowest row among equidistant points).  win_a[d] uint32 [n_d], grid
 * sets: the winning sample's composition a over the simplex's own vertices,
 * a_i in bits 8i..8i+7 (s* = sum_i (a_i/k) v_i; a face-inherited winner
 * carries zeros for the vertices it does not use; the interior sample with
 * the lowest rank in lexicographically descending composition order wins
 * exact ties, and the first attaining facet when the value comes from a
 * face).  Random sets: q, the winning sample's index within the simplex that
 * owns it, in bits 0..27, and in bits 28+i whether vertex i of this simplex
 * is a vertex of that owner (the simplex itself, or the face it inherits
 * from); the own sample with the lowest q wins ties among own samples, the
 * own samples win a tie with the facets, else the first attaining facet.
 * win_w[d] float [n_d][4] or NULL (required by the backward for random
 * sets): the winning sample's barycentric weights over the simplex's own
 * vertices, s* = sum_i w_i v_i (zeros for vertices the owner lacks).
 * evals: device uint64 [1] or NULL; receives (+=) the number of sample-point
 * distance evaluations executed for live samples.
 * tile_events: optional caller-created hipEvent_t handles; entries 3d,
 * 3d+1 and 3d+2 are recorded on `stream` before the cooperative tile search
 * of dimension d, between it and the per-sample search, and after the
 * per-sample search (NULL entries are skipped).  grid_events: the same, recorded
 * before and after the grid build.  For profiling only.
 * stats: device uint64 [32] or NULL; receives (+=), for dimension d,
 * [4d] ring steps (64 grid rows each) of the per-sample search, [4d+1]
 * samples handed to it, [4d+2] evaluations in the cooperative tile search,
 * [4d+3] evaluations in the per-sample search, [16+4d] sample slots the
 * tile search evaluated (live or not: its lane utilisation is [4d+2] over
 * this), [16+4d+1] the most ring steps of one per-sample search, [16+4d+2]
 * per-sample searches of more than 32 ring steps; [16+4d+3] is reserved
 * (zero). */
typedef struct {
    float *f[4];
    int32_t *win_x[4];
    uint32_t *win_a[4];
    uint64_t *evals;
    void *tile_events[12];
    uint64_t *stats;
    void *grid_events[2];
    float *win_w[4];
} flood_outputs;

/* Tuning knobs; pass NULL for the defaults (a zero field also selects its
 * default).  They change speed, never the values: cells_per_point (target
 * uniform-grid cells per point, 0.05..64), samples_per_lane (1, 2 or 4),
 * waves_per_block (1..4), tile_shells (cell shells a wave scans
 * cooperatively around its samples before handing open samples to the
 * per-sample search, 1..32, default 6; -1 sends every sample to the
 * per-sample search),
 * tile_extent (a tile whose samples span more cells than this along an axis
 * skips the cooperative search, 2..64, default 24),
 * queue_grab (open samples a wave of the per-sample search takes from the
 * queue per atomic: 1, 2, 4 or 8; default 4 when a dimension hands more
 * than 2^19 samples to that search, else 1),
 * tile_lanes (samples per tile of the cooperative search with
 * samples_per_lane 1: 64, 32 or 16; with fewer than 64 each sample is held
 * by 64/tile_lanes lanes that split every staged pass, so a tile covers a
 * smaller region; 0 selects the per-dimension default). */
typedef struct {
    float cells_per_point;
    int32_t samples_per_lane;
    int32_t waves_per_block;
    int32_t tile_shells;
    int32_t tile_extent;
    int32_t queue_grab;
    int32_t tile_lanes;
} flood_tuning;

size_t flood_filtration_workspace_size(const flood_problem *pb, const flood_tuning *tune);
flood_status flood_filtration(const flood_problem *pb, const flood_tuning *tune,
                              const flood_outputs *out, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * flood_filtration without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array
 * of FLOOD_STATIC_SCRATCH_BYTES on every device the library runs on, held
 * until the process ends; the call itself allocates nothing.  Arguments,
 * results and errors are those of flood_filtration; FLOOD_ENOMEM (before any
 * launch) when flood_filtration_workspace_size(pb, tune) exceeds the array --
 * about 580k points at L = N/100 and k = 6.  Every call on a device uses that
 * device's one array and leaves its contents behind (each call initialises
 * what it reads), so calls that overlap on one device -- on different
 * streams or threads -- race and must be serialised by the caller.
 */
#define FLOOD_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
flood_status flood_filtration_noalloc(const flood_problem *pb, const flood_tuning *tune,
                                      const flood_outputs *out, void *stream);

/* ---------------------------------------------------------------------------
 * Backward of loss(f) through (1), using the winners of a forward call.
 * Away from ties, f(sigma) = ||s* - x*|| with s* = sum_i w_i v_i (grid sets:
 * w_i = a_i/k from win_a; random sets: win_w, which must then be given), so
 * with u = (s* - x*)/||s* - x*|| (u = 0 when f = 0):
 *     grad_X[x*]  -= g u,      grad_L[v_i] += g w_i u,
 * g = grad_f[d][sigma].  grad_X [sum N][3] and grad_L [sum L][3] (device)
 * are accumulated into (+=); the caller zeroes them.  Uses float atomics,
 * so the summation order (not the terms) varies between runs.
 *   grad_f[d] device float [n_d] or NULL (treated as zero).
 */
flood_status flood_filtration_backward(const flood_problem *pb, const flood_outputs *fwd,
                                       const float *const grad_f[4], float *grad_X,
                                       float *grad_L, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FLOOD_H */
