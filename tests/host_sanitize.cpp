// Host-code driver for AddressSanitizer and UndefinedBehaviorSanitizer runs
// of the library's host entry points: the exact-predicate Delaunay
// triangulations (3-D and planar) and the Z/2 persistence reduction.  It
// feeds them random sets, integer lattices (every in-sphere test a tie, so
// the exact fallbacks run), near-degenerate perturbations of the lattices
// and degenerate sets that must be refused, exports every complex, builds a
// monotone filtration on it and reduces it.  Exit status 0 and "ok" on the
// last line when every call behaved; any sanitizer report aborts the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../include/flood.h"

namespace flood_host {
// the library's error sink (defined by the device-side translation unit in
// the full library); here it only keeps the last message
static std::string g_last;
void set_error(const std::string &msg) { g_last = msg; }
}  // namespace flood_host

static int failures = 0;
static long built = 0, refused = 0, fallbacks = 0;

static void check(bool ok, const char *what) {
    if (!ok) {
        std::printf("FAIL: %s (%s)\n", what, flood_host::g_last.c_str());
        ++failures;
    }
}

// a monotone filtration on an exported complex, reduced and exported
static void persistence_of(const std::vector<int64_t> &n, const std::vector<int32_t> &edges,
                           const std::vector<int32_t> &tri_edges, const std::vector<int32_t> &tet_tris,
                           std::mt19937 &rng) {
    std::uniform_real_distribution<float> u(0.f, 1.f);
    std::vector<float> f[4];
    f[0].assign(n[0], 0.f);
    f[1].resize(n[1]);
    for (int64_t e = 0; e < n[1]; ++e) f[1][e] = u(rng);
    f[2].resize(n[2]);
    for (int64_t t = 0; t < n[2]; ++t) {
        float m = u(rng);
        for (int i = 0; i < 3; ++i) m = std::fmax(m, f[1][tri_edges[3 * t + i]]);
        f[2][t] = m;
    }
    f[3].resize(n[3]);
    for (int64_t t = 0; t < n[3]; ++t) {
        float m = u(rng) < 0.3f ? 0.f : u(rng);  // ties with faces too
        for (int i = 0; i < 4; ++i) m = std::fmax(m, f[2][tet_tris[4 * t + i]]);
        f[3][t] = m;
    }
    const int64_t nn[4] = {n[0], n[1], n[2], n[3]};
    const float *fp[4] = {f[0].data(), f[1].data(), f[2].data(), f[3].data()};
    flood_diagram *dg = nullptr;
    check(flood_persistence(nn, edges.data(), tri_edges.data(), tet_tris.data(), fp, &dg) ==
              FLOOD_OK, "persistence");
    if (!dg) return;
    int64_t cnt[3];
    check(flood_diagram_counts(dg, cnt) == FLOOD_OK, "diagram counts");
    check(cnt[0] >= 1, "one essential component at least");
    for (int p = 0; p < 3; ++p) {
        std::vector<float> b(cnt[p]), d(cnt[p]);
        std::vector<int64_t> br(cnt[p]), dr(cnt[p]);
        check(flood_diagram_export(dg, p, b.data(), d.data(), br.data(), dr.data()) == FLOOD_OK, "diagram export");
        for (int64_t i = 0; i < cnt[p]; ++i) check(!(d[i] < b[i]), "death before birth");
    }
    flood_diagram_free(dg);
}

// triangulate, export, check the counts' Euler characteristic and reduce
static void run(const std::vector<float> &pts, int dim, bool expect_ok, std::mt19937 &rng, const char *what) {
    const int32_t L = (int32_t)(pts.size() / dim);
    flood_complex *cx = nullptr;
    const flood_status st = dim == 3 ? flood_delaunay(pts.data(), L, &cx) : flood_delaunay2d(pts.data(), L, &cx);
    if (!expect_ok) {
        check(st != FLOOD_OK && cx == nullptr, what);
        return;
    }
    if (st == FLOOD_EDEGENERATE) {  // an exactly cospherical set may be refused
        ++refused;
        return;
    }
    check(st == FLOOD_OK && cx != nullptr, what);
    if (!cx) return;
    int64_t c[5];
    check(flood_complex_counts(cx, c) == FLOOD_OK, "complex counts");
    ++built;
    fallbacks += c[4];
    const int64_t chi = c[0] - c[1] + c[2] - c[3];
    check(chi == 1, "Euler characteristic of a triangulated ball or disk");
    std::vector<int32_t> edges(2 * c[1]), tris(3 * c[2]), tets(4 * c[3] + 1), te(3 * c[2]), tt(4 * c[3] + 1);
    check(flood_complex_export(cx, edges.data(), tris.data(), tets.data(), te.data(), tt.data()) == FLOOD_OK,
          "complex export");
    flood_complex_free(cx);
    persistence_of({c[0], c[1], c[2], c[3]}, edges, te, tt, rng);
}

int main() {
    std::mt19937 rng(20260101);
    std::uniform_real_distribution<float> u(-1.f, 1.f);
    for (int trial = 0; trial < 40; ++trial) {
        const int L = 5 + (int)(rng() % 300);
        std::vector<float> p3(3 * L), p2(2 * L);
        for (auto &v : p3) v = u(rng);
        for (auto &v : p2) v = u(rng);
        run(p3, 3, true, rng, "random 3-D set");
        run(p2, 2, true, rng, "random planar set");
    }
    for (int m = 2; m <= 6; ++m) {  // lattices: every empty-sphere test is a tie
        std::vector<float> p3, p2;
        for (int x = 0; x < m; ++x)
            for (int y = 0; y < m; ++y) {
                p2.push_back((float)x);
                p2.push_back((float)y);
                for (int z = 0; z < m; ++z) {
                    p3.push_back((float)x);
                    p3.push_back((float)y);
                    p3.push_back((float)z);
                }
            }
        run(p3, 3, true, rng, "3-D lattice");
        run(p2, 2, true, rng, "planar lattice");
        for (auto &v : p3) v += 1e-6f * u(rng);  // near-degenerate: the filters fail, exact arithmetic decides
        for (auto &v : p2) v += 1e-6f * u(rng);
        run(p3, 3, true, rng, "perturbed 3-D lattice");
        run(p2, 2, true, rng, "perturbed planar lattice");
    }
    // sets that must be refused: too few points, coplanar / collinear, duplicates, NaN
    run({0, 0, 0, 1, 0, 0, 0, 1, 0}, 3, false, rng, "three points");
    run({0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0, 2, 3, 0}, 3, false, rng, "coplanar set");
    run({0, 0, 1, 1, 2, 2, 3, 3}, 2, false, rng, "collinear set");
    run({0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 1, 0, 0}, 3, false, rng, "duplicate point");
    run({0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, NAN}, 3, false, rng, "NaN coordinate");
    std::printf("complexes %ld, refused as cospherical %ld, exact fallbacks %ld\n", built, refused, fallbacks);
    std::printf(failures ? "failures %d\n" : "ok\n", failures);
    return failures ? 1 : 0;
}
