/*
 * CPU oracle for the flooding path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct loops.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the
 * product path never does.  Nothing here is shared with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * -ffp-contract=off matters: the landmark recipe below is specified op by op
 * in IEEE single precision and must not be fused into FMAs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Farthest-point sampling (greedy k-centre; Sec. 2 "Theoretical results",
 * the 2-approximation of the covering radius).  Recipe, all in float32:
 *   dx = x - l (one rounding), d2 = (dx*dx + dy*dy) + dz*dz (each op rounded,
 *   no FMA), mind_i = min(mind_i, d2), next = argmax mind (lowest index on
 *   ties).  mind starts as the distance to the start point.
 * radius[t] = sqrtf(max_i mind_i) after landmarks 0..t are chosen, i.e. the
 * covering radius d_H(X, {l_0..l_t}); radius[L-1] is d_H(X, L).
 * Returns 0, or 4 if fewer than L distinct points exist.
 */
static float fps_d2(const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    float sx = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    float s = sx + sy;
    return s + sz;
}

int or_fps(const float *X, int64_t N, int64_t start, int32_t L,
           int32_t *idx, float *radius, int nthreads)
{
    if (N <= 0 || L <= 0 || L > N || start < 0 || start >= N)
        return 1;
    float *mind = (float *)malloc(sizeof(float) * (size_t)N);
    if (!mind)
        return 2;
    idx[0] = (int32_t)start;
    const float *l = X + 3 * start;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < N; ++i)
        mind[i] = fps_d2(X + 3 * i, l);
    int rc = 0;
    for (int32_t t = 1; t <= L; ++t) {
        /* argmax with lowest index on ties */
        float best = -1.0f;
        int64_t besti = -1;
#pragma omp parallel num_threads(nthreads)
        {
            float tb = -1.0f;
            int64_t ti = -1;
#pragma omp for schedule(static) nowait
            for (int64_t i = 0; i < N; ++i) {
                if (mind[i] > tb) {
                    tb = mind[i];
                    ti = i;
                }
            }
#pragma omp critical
            {
                if (tb > best || (tb == best && ti >= 0 && ti < besti)) {
                    best = tb;
                    besti = ti;
                }
            }
        }
        radius[t - 1] = sqrtf(best);
        if (t == L)
            break;
        if (!(best > 0.0f)) {
            rc = 4;
            break;
        }
        idx[t] = (int32_t)besti;
        l = X + 3 * besti;
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            float d2 = fps_d2(X + 3 * i, l);
            if (d2 < mind[i])
                mind[i] = d2;
        }
    }
    free(mind);
    return rc;
}

/* ------------------------------------------------------------------------
 * Sampled flood values (Sec. 4.1, the sampled complex Flood_r(X,L,P) with
 * the barycentric grid of Lemma 6):
 *   P_sigma = { sum_i (a_i/k) v_i : a_i >= 0 integers, sum_i a_i = k }
 *   f_P(sigma) = max_{p in P_sigma} min_{x in X} ||p - x||
 * in double precision, distances by direct difference.  Samples are visited
 * with the composition a in lexicographically descending order, starting at
 * (k,0,..,0); the winner a* is the first sample attaining the maximum, and x*
 * the lowest index attaining the minimum.
 *
 * gap_s / gap_x (optional): the gap between the best and second-best sample
 * value, and at the best sample between its nearest and second-nearest
 * point -- small gaps mark simplices whose winner is nearly tied (in masked
 * mode the second-nearest point is taken within the mask).
 *
 * mode 0 (brute): min over all of X.
 * mode 1 (masked): min over X cap B(c, rho) with c the midpoint of the
 *   longest edge, r = max_i ||c - v_i|| and rho = sqrt(2) r (rho = r for an
 *   edge, rho = 0 for a vertex), widened by a factor (1 + 1e-12).  This is
 *   the enclosing-ball mask of Lemma 7, exact when every landmark is a point
 *   of X.  The candidates are found as the paper's appendix describes: X is
 *   presorted along the first axis (xs, order), a binary search yields the
 *   slice |x - c_x| <= rho, and the ball test filters the slice.
 *
 * Sample coordinates: p = 0; for i in 0..d: p += (a_i/k) * v_i with
 * v_i the landmark coordinate, so a face's samples are bit-identical
 * to the coface samples that carry zeros in the extra positions.
 */
static void next_composition_desc(int *a, int d, int *done)
{
    /* Successor of a (d+1 non-negative parts, fixed sum) in lexicographically
       descending order: take the rightmost j <= d-1 with a[j] > 0, move one
       unit from a[j] to a[j+1] and gather the whole tail a[j+1..d] there. */
    int j = d - 1;
    while (j >= 0 && a[j] == 0)
        --j;
    if (j < 0) {
        *done = 1;
        return;
    }
    int tail = 0;
    for (int i = j + 1; i <= d; ++i) {
        tail += a[i];
        a[i] = 0;
    }
    a[j] -= 1;
    a[j + 1] = tail + 1;
}

static double dist2(const double *p, const double *x)
{
    double dx = p[0] - x[0];
    double dy = p[1] - x[1];
    double dz = p[2] - x[2];
    return dx * dx + dy * dy + dz * dz;
}

/* Inputs are double so that finite-difference probes can move points by
   less than a float32 ulp; float32 data converts to double exactly. */
int or_flood(const double *X, int64_t N, const double *Lxyz,
             const int32_t *simp, int64_t n, int32_t d, int32_t k,
             int32_t mode, const double *xs, const int64_t *order,
             double *f, int32_t *win_a, int32_t *win_x, int64_t *evals_out, double *gap_s,
             double *gap_x, int nthreads)
{
    if (d < 0 || d > 3 || k < 1 || N <= 0)
        return 1;
    int rc = 0;
    int64_t evals = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : evals)
    {
        int64_t *cand = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < n; ++s) {
            double v[4][3];
            for (int i = 0; i <= d; ++i)
                for (int c = 0; c < 3; ++c)
                    v[i][c] = Lxyz[3 * (int64_t)simp[s * (d + 1) + i] + c];
            /* candidate set */
            int64_t nc = N;
            if (mode == 1) {
                double c0[3] = {v[0][0], v[0][1], v[0][2]};
                double rho = 0.0;
                if (d >= 1) {
                    int bi = 0, bj = 1;
                    double bl = -1.0;
                    for (int i = 0; i <= d; ++i)
                        for (int j = i + 1; j <= d; ++j) {
                            double e[3] = {v[i][0] - v[j][0], v[i][1] - v[j][1], v[i][2] - v[j][2]};
                            double l2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                            if (l2 > bl) {
                                bl = l2;
                                bi = i;
                                bj = j;
                            }
                        }
                    for (int c = 0; c < 3; ++c)
                        c0[c] = 0.5 * (v[bi][c] + v[bj][c]);
                    double r = 0.0;
                    for (int i = 0; i <= d; ++i) {
                        double e[3] = {v[i][0] - c0[0], v[i][1] - c0[1], v[i][2] - c0[2]};
                        double ri = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                        if (ri > r)
                            r = ri;
                    }
                    rho = (d == 1) ? r : sqrt(2.0) * r;
                }
                rho *= (1.0 + 1e-12);
                /* slice along the first axis by binary search */
                double lo = c0[0] - rho, hi = c0[0] + rho;
                int64_t a = 0, b = N;
                while (a < b) {
                    int64_t m = (a + b) / 2;
                    if (xs[3 * m] < lo)
                        a = m + 1;
                    else
                        b = m;
                }
                int64_t first = a;
                a = first;
                b = N;
                while (a < b) {
                    int64_t m = (a + b) / 2;
                    if (xs[3 * m] <= hi)
                        a = m + 1;
                    else
                        b = m;
                }
                int64_t last = a;
                nc = 0;
                for (int64_t m = first; m < last; ++m) {
                    if (dist2(c0, xs + 3 * m) <= rho * rho) {
                        if (nc == cap) {
                            cap = cap ? 2 * cap : 1024;
                            cand = (int64_t *)realloc(cand, sizeof(int64_t) * (size_t)cap);
                        }
                        cand[nc++] = order[m];
                    }
                }
            }
            /* samples in lexicographically descending composition order */
            int a[4] = {0, 0, 0, 0};
            a[0] = k;
            int done = 0;
            double fbest = -1.0, fsecond = -1.0, xgap = INFINITY;
            int abest[4] = {0, 0, 0, 0};
            int64_t xbest = -1;
            while (!done) {
                double p[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i <= d; ++i) {
                    double w = (double)a[i] / (double)k;
                    p[0] += w * v[i][0];
                    p[1] += w * v[i][1];
                    p[2] += w * v[i][2];
                }
                double m2 = INFINITY, m2b = INFINITY;  /* nearest and second nearest */
                int64_t mi = -1;
                evals += nc;
                for (int64_t t = 0; t < nc; ++t) {
                    int64_t xi = (mode == 1) ? cand[t] : t;
                    double q = dist2(p, X + 3 * xi);
                    if (q < m2 || (q == m2 && xi < mi)) {
                        m2b = m2;
                        m2 = q;
                        mi = xi;
                    } else if (q < m2b) {
                        m2b = q;
                    }
                }
                double dist = sqrt(m2);
                if (mi < 0) {
#pragma omp atomic write
                    rc = 5; /* empty candidate set: mask precondition violated */
                }
                if (dist > fbest) {
                    fsecond = fbest;
                    fbest = dist;
                    xbest = mi;
                    xgap = sqrt(m2b) - dist;
                    for (int i = 0; i < 4; ++i)
                        abest[i] = a[i];
                } else if (dist > fsecond) {
                    fsecond = dist;
                }
                if (d == 0)
                    break;
                next_composition_desc(a, d, &done);
            }
            f[s] = fbest;
            if (gap_s)
                gap_s[s] = fsecond < 0.0 ? INFINITY : fbest - fsecond;
            if (gap_x)
                gap_x[s] = xgap;
            win_x[s] = (int32_t)xbest;
            for (int i = 0; i < 4; ++i)
                win_a[4 * s + i] = abest[i];
        }
        free(cand);
    }
    if (evals_out)
        *evals_out += evals;
    return rc;
}

/* number of threads OpenMP will use by default (for reporting) */
#include <omp.h>
int or_max_threads(void) { return omp_get_max_threads(); }

/* Number of samples the enumeration above visits for a d-simplex at k
   segments per edge (a pin: it must be the size of the grid of Lemma 6,
   C(k+d, d)); also writes them (row-major, d+1 ints each) if out != NULL. */
int64_t or_count_samples(int32_t d, int32_t k, int32_t *out)
{
    int a[4] = {0, 0, 0, 0};
    a[0] = k;
    int done = 0;
    int64_t c = 0;
    while (!done) {
        if (out)
            for (int i = 0; i <= d; ++i)
                out[c * (d + 1) + i] = a[i];
        ++c;
        if (d == 0)
            break;
        next_composition_desc(a, d, &done);
    }
    return c;
}

/* ------------------------------------------------------------------------
 * Random sample sets (Thm. 5 allows any P_sigma inside conv sigma; Lemma 9:
 * points drawn uniformly from conv sigma).  The draws are specified by a
 * counter-based generator so that the library and this oracle produce the
 * same sets from their own code: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011), written here
 * from that definition.  Sample q of the simplex in (cloud-local) row r of
 * dimension d: counter (q, r, d, 0), key (seed, 0); u_i = (word_i >> 40) *
 * 2^-24 for i < d; sorted u_(1) <= ... <= u_(d), the barycentric weights
 * are the spacings u_(1), u_(2) - u_(1), ..., 1 - u_(d) (uniform on the
 * simplex: the spacings of sorted uniforms are Dirichlet(1, ..., 1)).
 */
static void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        unsigned __int128 p0 = (unsigned __int128)m0 * c[0];
        unsigned __int128 p1 = (unsigned __int128)m1 * c[2];
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c[1] ^ k0;
        uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

/* the raw generator, for pinning against an independent implementation */
void or_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out)
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    philox4x64_10(c, key[0], key[1]);
    for (int i = 0; i < 4; ++i)
        out[i] = c[i];
}

void or_random_weights(int32_t d, int64_t q, int64_t row, uint64_t seed, double *w)
{
    if (d == 0) {
        w[0] = 1.0;
        return;
    }
    uint64_t c[4] = {(uint64_t)q, (uint64_t)row, (uint64_t)d, 0};
    philox4x64_10(c, seed, 0);
    double u[3];
    for (int i = 0; i < d; ++i)
        u[i] = (double)(c[i] >> 40) / 16777216.0;
    /* insertion sort of the d <= 3 uniforms */
    for (int i = 1; i < d; ++i)
        for (int j = i; j > 0 && u[j] < u[j - 1]; --j) {
            double t = u[j];
            u[j] = u[j - 1];
            u[j - 1] = t;
        }
    w[0] = u[0];
    for (int i = 1; i < d; ++i)
        w[i] = u[i] - u[i - 1];
    w[d] = 1.0 - u[d - 1];
}

/* Lemma 7 candidate set for a simplex with vertices v[0..d] (same reading
   as or_flood: centre at the midpoint of the longest edge, radius sqrt(2)
   times the enclosing radius, the half edge for an edge), gathered from the
   x-presorted copy. */
static int64_t lemma7_candidates(const double v[4][3], int d, int64_t N, const double *xs, const int64_t *order,
                                 int64_t **cand, int64_t *cap)
{
    double c0[3] = {v[0][0], v[0][1], v[0][2]};
    double rho = 0.0;
    if (d >= 1) {
        int bi = 0, bj = 1;
        double bl = -1.0;
        for (int i = 0; i <= d; ++i)
            for (int j = i + 1; j <= d; ++j) {
                double e[3] = {v[i][0] - v[j][0], v[i][1] - v[j][1], v[i][2] - v[j][2]};
                double l2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                if (l2 > bl) {
                    bl = l2;
                    bi = i;
                    bj = j;
                }
            }
        for (int c = 0; c < 3; ++c)
            c0[c] = 0.5 * (v[bi][c] + v[bj][c]);
        double r = 0.0;
        for (int i = 0; i <= d; ++i) {
            double e[3] = {v[i][0] - c0[0], v[i][1] - c0[1], v[i][2] - c0[2]};
            double ri = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            if (ri > r)
                r = ri;
        }
        rho = (d == 1) ? r : sqrt(2.0) * r;
    }
    rho *= (1.0 + 1e-12);
    double lo = c0[0] - rho, hi = c0[0] + rho;
    int64_t a = 0, b = N;
    while (a < b) {
        int64_t m = (a + b) / 2;
        if (xs[3 * m] < lo)
            a = m + 1;
        else
            b = m;
    }
    int64_t first = a;
    a = first;
    b = N;
    while (a < b) {
        int64_t m = (a + b) / 2;
        if (xs[3 * m] <= hi)
            a = m + 1;
        else
            b = m;
    }
    int64_t last = a, nc = 0;
    for (int64_t m = first; m < last; ++m) {
        if (dist2(c0, xs + 3 * m) <= rho * rho) {
            if (nc == *cap) {
                *cap = *cap ? 2 * *cap : 1024;
                *cand = (int64_t *)realloc(*cand, sizeof(int64_t) * (size_t)*cap);
            }
            (*cand)[nc++] = order[m];
        }
    }
    return nc;
}

/* Own value of each simplex under random sample sets: the max over its m
   random samples (vertices: the vertex) of the distance to X, without the
   face closure.  rows[s] is the simplex's row within its cloud (the
   generator's counter).  Winner: the first sample in q order attaining the
   max, its nearest point the lowest index.  mode 0 brute, 1 Lemma 7 mask. */
int or_flood_random(const double *X, int64_t N, const double *Lxyz, const int32_t *simp, const int64_t *rows,
                    int64_t n, int32_t d, int32_t m, uint64_t seed, int32_t mode, const double *xs,
                    const int64_t *order, double *f, int32_t *win_q, int32_t *win_x, int64_t *evals_out,
                    int nthreads)
{
    if (d < 0 || d > 3 || m < 1 || N <= 0)
        return 1;
    int rc = 0;
    int64_t evals = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : evals)
    {
        int64_t *cand = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < n; ++s) {
            double v[4][3] = {{0.0}};
            for (int i = 0; i <= d; ++i)
                for (int c = 0; c < 3; ++c)
                    v[i][c] = Lxyz[3 * (int64_t)simp[s * (d + 1) + i] + c];
            int64_t nc = mode == 1 ? lemma7_candidates(v, d, N, xs, order, &cand, &cap) : N;
            int nq = d == 0 ? 1 : m;
            double fbest = -1.0;
            int32_t qbest = 0;
            int64_t xbest = -1;
            for (int q = 0; q < nq; ++q) {
                double w[4];
                or_random_weights(d, q, rows[s], seed, w);
                double p[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i <= d; ++i)
                    for (int c = 0; c < 3; ++c)
                        p[c] += w[i] * v[i][c];
                double m2 = INFINITY;
                int64_t mi = -1;
                evals += nc;
                for (int64_t t = 0; t < nc; ++t) {
                    int64_t xi = mode == 1 ? cand[t] : t;
                    double dd = dist2(p, X + 3 * xi);
                    if (dd < m2 || (dd == m2 && xi < mi)) {
                        m2 = dd;
                        mi = xi;
                    }
                }
                if (mi < 0) {
#pragma omp atomic write
                    rc = 5;
                }
                double dist = sqrt(m2);
                if (dist > fbest) {
                    fbest = dist;
                    qbest = q;
                    xbest = mi;
                }
            }
            f[s] = fbest;
            win_q[s] = qbest;
            win_x[s] = (int32_t)xbest;
        }
        free(cand);
    }
    if (evals_out)
        *evals_out += evals;
    return rc;
}
