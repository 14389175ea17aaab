// Delaunay triangulation of the landmarks on the host (the simplex set of
// the Flood complex is Del(L), Sec. 4).  Incremental Bowyer-Watson
// insertion in Morton order with a symbolic infinite vertex for the hull.
//
// Predicates: orient(a,b,c,d) = det[a-d; b-d; c-d]; insph(a,b,c,d,e) = det of
// the rows (p - e, |p - e|^2), p in (a,b,c,d); e is strictly inside the
// circumsphere of a positively oriented (a,b,c,d) iff insph > 0.  Both are
// evaluated in FP64 with a loose static error filter; undecided cases are
// recomputed exactly with integers (every float32 is an integer times a
// power of two), so the triangulation is the exact Delaunay triangulation of
// the float32 input.  An exact zero that decides the result (coplanar or
// cospherical configurations) is reported as degenerate input.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/flood.h"

namespace flood_host {
void set_error(const std::string &msg);
}

namespace {

// ---------------------------------------------------------------------------
// minimal signed big integer (sign + magnitude, base 2^32)
struct Big {
    int sign = 0;                 // -1, 0, +1
    std::vector<uint32_t> mag;    // little endian, no leading zeros

    static Big from_u64_shift(uint64_t m, int shift, int sgn) {
        Big r;
        if (m == 0) return r;
        r.sign = sgn;
        int limb = shift / 32, bit = shift % 32;
        r.mag.assign(limb, 0u);
        unsigned __int128 v = (unsigned __int128)m << bit;
        while (v) {
            r.mag.push_back((uint32_t)v);
            v >>= 32;
        }
        return r;
    }
    static int cmp_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
        for (size_t i = a.size(); i-- > 0;)
            if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
        return 0;
    }
    static std::vector<uint32_t> add_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
        std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0u);
        uint64_t c = 0;
        for (size_t i = 0; i < r.size(); ++i) {
            uint64_t s = c + (i < a.size() ? a[i] : 0u) + (i < b.size() ? b[i] : 0u);
            r[i] = (uint32_t)s;
            c = s >> 32;
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    static std::vector<uint32_t> sub_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {  // |a|>=|b|
        std::vector<uint32_t> r(a.size(), 0u);
        int64_t br = 0;
        for (size_t i = 0; i < a.size(); ++i) {
            int64_t s = (int64_t)a[i] - (i < b.size() ? (int64_t)b[i] : 0) - br;
            br = s < 0;
            r[i] = (uint32_t)(s + (br ? ((int64_t)1 << 32) : 0));
        }
        while (!r.empty() && r.back() == 0) r.pop_back();
        return r;
    }
    friend Big operator+(const Big &a, const Big &b) {
        if (a.sign == 0) return b;
        if (b.sign == 0) return a;
        Big r;
        if (a.sign == b.sign) {
            r.mag = add_mag(a.mag, b.mag);
            r.sign = a.sign;
        } else {
            int c = cmp_mag(a.mag, b.mag);
            if (c == 0) return r;
            if (c > 0) {
                r.mag = sub_mag(a.mag, b.mag);
                r.sign = a.sign;
            } else {
                r.mag = sub_mag(b.mag, a.mag);
                r.sign = b.sign;
            }
        }
        return r;
    }
    Big neg() const {
        Big r = *this;
        r.sign = -r.sign;
        return r;
    }
    friend Big operator-(const Big &a, const Big &b) { return a + b.neg(); }
    friend Big operator*(const Big &a, const Big &b) {
        Big r;
        if (a.sign == 0 || b.sign == 0) return r;
        std::vector<uint64_t> acc(a.mag.size() + b.mag.size() + 1, 0);
        r.mag.assign(a.mag.size() + b.mag.size() + 1, 0u);
        for (size_t i = 0; i < a.mag.size(); ++i) {
            uint64_t c = 0;
            for (size_t j = 0; j < b.mag.size(); ++j) {
                uint64_t cur = (uint64_t)r.mag[i + j] + (uint64_t)a.mag[i] * b.mag[j] + c;
                r.mag[i + j] = (uint32_t)cur;
                c = cur >> 32;
            }
            size_t k = i + b.mag.size();
            while (c) {
                uint64_t cur = (uint64_t)r.mag[k] + c;
                r.mag[k] = (uint32_t)cur;
                c = cur >> 32;
                ++k;
            }
        }
        while (!r.mag.empty() && r.mag.back() == 0) r.mag.pop_back();
        r.sign = r.mag.empty() ? 0 : a.sign * b.sign;
        return r;
    }
};

// float32 value as (integer mantissa, exponent): v = m * 2^e
struct Fx {
    int64_t m;
    int e;
};
Fx decompose(float v) {
    if (v == 0.0f) return {0, 0};
    int e;
    float fr = std::frexp(v, &e);             // v = fr * 2^e, 0.5 <= |fr| < 1
    int64_t m = (int64_t)std::ldexp((double)fr, 24);  // exact: 24-bit mantissa
    return {m, e - 24};
}

struct ExactCoords {
    // integer coordinates of up to 5 points at a common scale 2^E
    Big c[5][3];
};

ExactCoords exact_scale(const float *const *p, int npts) {
    int E = 1 << 30;
    Fx f[5][3];
    for (int i = 0; i < npts; ++i)
        for (int a = 0; a < 3; ++a) {
            f[i][a] = decompose(p[i][a]);
            if (f[i][a].m != 0) E = std::min(E, f[i][a].e);
        }
    ExactCoords r;
    for (int i = 0; i < npts; ++i)
        for (int a = 0; a < 3; ++a) {
            int64_t m = f[i][a].m;
            if (m == 0) continue;
            uint64_t um = (uint64_t)(m < 0 ? -m : m);
            r.c[i][a] = Big::from_u64_shift(um, f[i][a].e - E, m < 0 ? -1 : 1);
        }
    return r;
}

Big det3(const Big A[3], const Big B[3], const Big C[3]) {
    return A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) + A[2] * (B[0] * C[1] - B[1] * C[0]);
}

int orient_exact(const float *a, const float *b, const float *c, const float *d) {
    const float *p[4] = {a, b, c, d};
    ExactCoords x = exact_scale(p, 4);
    Big A[3], B[3], C[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = x.c[0][k] - x.c[3][k];
        B[k] = x.c[1][k] - x.c[3][k];
        C[k] = x.c[2][k] - x.c[3][k];
    }
    return det3(A, B, C).sign;
}

int insph_exact(const float *a, const float *b, const float *c, const float *d, const float *e) {
    const float *p[5] = {a, b, c, d, e};
    ExactCoords x = exact_scale(p, 5);
    Big R[4][3], W[4];
    for (int i = 0; i < 4; ++i) {
        for (int k = 0; k < 3; ++k) R[i][k] = x.c[i][k] - x.c[4][k];
        W[i] = R[i][0] * R[i][0] + R[i][1] * R[i][1] + R[i][2] * R[i][2];
    }
    Big v = (W[0] * det3(R[1], R[2], R[3])).neg() + W[1] * det3(R[0], R[2], R[3]) - W[2] * det3(R[0], R[1], R[3]) +
            W[3] * det3(R[0], R[1], R[2]);
    return v.sign;
}

struct Predicates {
    int64_t fallbacks = 0;

    int orient(const float *a, const float *b, const float *c, const float *d) {
        const double ax = (double)a[0] - d[0], ay = (double)a[1] - d[1], az = (double)a[2] - d[2];
        const double bx = (double)b[0] - d[0], by = (double)b[1] - d[1], bz = (double)b[2] - d[2];
        const double cx = (double)c[0] - d[0], cy = (double)c[1] - d[1], cz = (double)c[2] - d[2];
        const double det = ax * (by * cz - bz * cy) - ay * (bx * cz - bz * cx) + az * (bx * cy - by * cx);
        const double perm = std::fabs(ax) * (std::fabs(by * cz) + std::fabs(bz * cy)) +
                            std::fabs(ay) * (std::fabs(bx * cz) + std::fabs(bz * cx)) +
                            std::fabs(az) * (std::fabs(bx * cy) + std::fabs(by * cx));
        if (std::fabs(det) > 1e-12 * perm) return det > 0 ? 1 : -1;
        ++fallbacks;
        return orient_exact(a, b, c, d);
    }

    static double d3(const double *A, const double *B, const double *C) {
        return A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) + A[2] * (B[0] * C[1] - B[1] * C[0]);
    }
    static double p3(const double *A, const double *B, const double *C) {
        return std::fabs(A[0]) * (std::fabs(B[1] * C[2]) + std::fabs(B[2] * C[1])) +
               std::fabs(A[1]) * (std::fabs(B[0] * C[2]) + std::fabs(B[2] * C[0])) +
               std::fabs(A[2]) * (std::fabs(B[0] * C[1]) + std::fabs(B[1] * C[0]));
    }
    int insph(const float *a, const float *b, const float *c, const float *d, const float *e) {
        const float *p[4] = {a, b, c, d};
        double R[4][3], W[4];
        for (int i = 0; i < 4; ++i) {
            for (int k = 0; k < 3; ++k) R[i][k] = (double)p[i][k] - e[k];
            W[i] = R[i][0] * R[i][0] + R[i][1] * R[i][1] + R[i][2] * R[i][2];
        }
        const double det = -W[0] * d3(R[1], R[2], R[3]) + W[1] * d3(R[0], R[2], R[3]) - W[2] * d3(R[0], R[1], R[3]) +
                           W[3] * d3(R[0], R[1], R[2]);
        const double perm = W[0] * p3(R[1], R[2], R[3]) + W[1] * p3(R[0], R[2], R[3]) + W[2] * p3(R[0], R[1], R[3]) +
                            W[3] * p3(R[0], R[1], R[2]);
        if (std::fabs(det) > 1e-11 * perm) return det > 0 ? 1 : -1;
        ++fallbacks;
        return insph_exact(a, b, c, d, e);
    }
};

// ---------------------------------------------------------------------------
// triangulation with an infinite vertex (-1).  Every tet is positively
// oriented; for a tet containing the infinite vertex, replacing it by a point
// q gives a positive orientation iff q lies strictly beyond its hull facet.

constexpr int INF = -1;

struct Tet {
    int v[4];
    int n[4];  // neighbour across the face opposite v[i]
};

struct Degenerate {};

struct Triangulation {
    const float *P;
    Predicates pr;
    std::vector<Tet> t;
    std::vector<char> dead;
    std::vector<uint32_t> in_cav, tested;  // insertion id marks
    std::vector<int> free_list;
    // per-insertion buffers, kept across insertions (no allocation per point)
    struct EdgeSlot {
        uint64_t key;
        int tet, face;
    };
    std::vector<int> cavity, stack;
    std::vector<EdgeSlot> open_edges;
    uint32_t ins = 0;
    int last = 0;
    uint64_t rng = 0x9e3779b97f4a7c15ull;

    const float *pt(int i) const { return P + 3 * (size_t)i; }
    static bool infinite_v(const Tet &x) {
        return x.v[0] == INF || x.v[1] == INF || x.v[2] == INF || x.v[3] == INF;
    }
    bool infinite(int ti) const { return infinite_v(t[ti]); }
    int new_tet() {
        int i;
        if (!free_list.empty()) {
            i = free_list.back();
            free_list.pop_back();
        } else {
            t.push_back(Tet{});
            dead.push_back(0);
            in_cav.push_back(0);
            tested.push_back(0);
            i = (int)t.size() - 1;
        }
        dead[i] = 0;
        in_cav[i] = 0;
        tested[i] = 0;
        return i;
    }
    uint32_t rnd() {
        rng ^= rng << 13;
        rng ^= rng >> 7;
        rng ^= rng << 17;
        return (uint32_t)rng;
    }
    // orientation of tet ti with vertex slot i replaced by point q
    int orient_with(int ti, int i, int q) {
        const Tet &x = t[ti];
        const float *p[4];
        for (int k = 0; k < 4; ++k) p[k] = (k == i) ? pt(q) : pt(x.v[k]);
        return pr.orient(p[0], p[1], p[2], p[3]);
    }
    bool conflict(int ti, int q) {
        const Tet &x = t[ti];
        for (int k = 0; k < 4; ++k)
            if (x.v[k] == INF) {
                int o = orient_with(ti, k, q);
                if (o == 0) throw Degenerate();
                return o > 0;
            }
        int s = pr.insph(pt(x.v[0]), pt(x.v[1]), pt(x.v[2]), pt(x.v[3]), pt(q));
        if (s == 0) throw Degenerate();
        return s > 0;
    }
    int locate(int q) {
        int cur = last;
        size_t steps = 0, limit = 8 * t.size() + 64;
        while (steps++ < limit) {
            if (infinite(cur)) return cur;
            int start = (int)(rnd() & 3u);
            int moved = -1;
            for (int r = 0; r < 4; ++r) {
                int i = (start + r) & 3;
                if (orient_with(cur, i, q) < 0) {
                    moved = t[cur].n[i];
                    break;
                }
            }
            if (moved < 0) return cur;
            cur = moved;
        }
        // fallback: any live tet in conflict
        for (int i = 0; i < (int)t.size(); ++i)
            if (!dead[i] && conflict(i, q)) return i;
        throw Degenerate();
    }
    void insert(int q) {
        int c0 = locate(q);
        if (!conflict(c0, q)) throw Degenerate();
        ++ins;
        cavity.clear();
        stack.clear();
        stack.push_back(c0);
        in_cav[c0] = ins;
        tested[c0] = ins;
        while (!stack.empty()) {
            int c = stack.back();
            stack.pop_back();
            cavity.push_back(c);
            for (int i = 0; i < 4; ++i) {
                int nb = t[c].n[i];
                if (tested[nb] == ins) continue;
                tested[nb] = ins;
                if (conflict(nb, q)) {
                    in_cav[nb] = ins;
                    stack.push_back(nb);
                }
            }
        }
        // new tets on the cavity boundary; faces through q are glued by edge
        // (a cavity has a few dozen boundary faces: the still unmatched edges
        // are searched linearly)
        open_edges.clear();
        int created_finite = -1;
        for (int c : cavity) {
            for (int i = 0; i < 4; ++i) {
                int nb = t[c].n[i];
                if (in_cav[nb] == ins) continue;
                Tet x = t[c];
                x.v[i] = q;
                for (int k = 0; k < 4; ++k) x.n[k] = -1;
                x.n[i] = nb;
                if (!infinite_v(x)) {
                    if (pr.orient(pt(x.v[0]), pt(x.v[1]), pt(x.v[2]), pt(x.v[3])) <= 0) throw Degenerate();
                }
                int nt = new_tet();
                t[nt] = x;
                for (int k = 0; k < 4; ++k)
                    if (t[nb].n[k] == c) t[nb].n[k] = nt;
                if (created_finite < 0 && !infinite_v(x)) created_finite = nt;
                for (int j = 0; j < 4; ++j) {
                    if (j == i) continue;
                    int e0 = 0, e1 = 0, m = 0;
                    for (int k = 0; k < 4; ++k)
                        if (k != i && k != j) (m++ == 0 ? e0 : e1) = x.v[k];
                    int lo = std::min(e0, e1), hi = std::max(e0, e1);
                    uint64_t key = ((uint64_t)(uint32_t)(lo + 1) << 32) | (uint32_t)(hi + 1);
                    size_t at = 0;
                    while (at < open_edges.size() && open_edges[at].key != key) ++at;
                    if (at == open_edges.size()) {
                        open_edges.push_back(EdgeSlot{key, nt, j});
                    } else {
                        t[nt].n[j] = open_edges[at].tet;
                        t[open_edges[at].tet].n[open_edges[at].face] = nt;
                        open_edges[at] = open_edges.back();
                        open_edges.pop_back();
                    }
                }
            }
        }
        if (!open_edges.empty()) throw Degenerate();
        for (int c : cavity) {
            dead[c] = 1;
            free_list.push_back(c);
        }
        if (created_finite >= 0) last = created_finite;
    }
};

uint64_t spread3(uint32_t x) {
    uint64_t v = x & 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

}  // namespace

struct flood_complex {
    int32_t L = 0;
    std::vector<std::array<int32_t, 2>> E;
    std::vector<std::array<int32_t, 3>> F;
    std::vector<std::array<int32_t, 4>> T;
    std::vector<std::array<int32_t, 3>> tri_edges;
    std::vector<std::array<int32_t, 4>> tet_tris;
    int64_t fallbacks = 0;
};

extern "C" flood_status flood_delaunay(const float *Lxyz, int32_t L, flood_complex **out) {
    using flood_host::set_error;
    if (!out) {
        set_error("flood_delaunay: out is NULL");
        return FLOOD_EINVAL;
    }
    *out = nullptr;
    if (!Lxyz || L < 0) {
        set_error("flood_delaunay: bad arguments");
        return FLOOD_EINVAL;
    }
    if (L < 4) {
        set_error("flood_delaunay: need at least 4 landmarks");
        return FLOOD_EDEGENERATE;
    }
    for (int64_t i = 0; i < 3 * (int64_t)L; ++i)
        if (!std::isfinite(Lxyz[i])) {
            set_error("flood_delaunay: non-finite coordinate");
            return FLOOD_EINVAL;
        }
    try {
        // duplicates
        std::vector<int32_t> ord(L);
        for (int32_t i = 0; i < L; ++i) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            return std::lexicographical_compare(Lxyz + 3 * (size_t)a, Lxyz + 3 * (size_t)a + 3, Lxyz + 3 * (size_t)b,
                                                Lxyz + 3 * (size_t)b + 3);
        });
        for (int32_t i = 1; i < L; ++i)
            if (std::memcmp(Lxyz + 3 * (size_t)ord[i], Lxyz + 3 * (size_t)ord[i - 1], 3 * sizeof(float)) == 0) {
                set_error("flood_delaunay: duplicate landmark coordinates");
                return FLOOD_EDEGENERATE;
            }
        // Morton insertion order
        float lo[3] = {Lxyz[0], Lxyz[1], Lxyz[2]}, hi[3] = {Lxyz[0], Lxyz[1], Lxyz[2]};
        for (int32_t i = 0; i < L; ++i)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], Lxyz[3 * (size_t)i + a]);
                hi[a] = std::max(hi[a], Lxyz[3 * (size_t)i + a]);
            }
        std::vector<std::pair<uint64_t, int32_t>> mk(L);
        for (int32_t i = 0; i < L; ++i) {
            uint64_t code = 0;
            for (int a = 0; a < 3; ++a) {
                double ext = (double)hi[a] - lo[a];
                double u = ext > 0 ? ((double)Lxyz[3 * (size_t)i + a] - lo[a]) / ext : 0.0;
                uint32_t q = (uint32_t)std::min(2097151.0, std::max(0.0, u * 2097151.0));
                code |= spread3(q) << a;
            }
            mk[i] = {code, i};
        }
        std::sort(mk.begin(), mk.end());
        Triangulation tr;
        tr.P = Lxyz;
        // first tetrahedron: 4 affinely independent points in insertion order
        std::vector<int32_t> seq(L);
        for (int32_t i = 0; i < L; ++i) seq[i] = mk[i].second;
        int32_t a0 = seq[0], a1 = -1, a2 = -1, a3 = -1;
        size_t ia1 = 0, ia2 = 0, ia3 = 0;
        for (size_t i = 1; i < seq.size() && a1 < 0; ++i) { a1 = seq[i]; ia1 = i; }
        // a2: not collinear with a0,a1 (some orientation with an auxiliary test)
        auto collinear = [&](int32_t p, int32_t q, int32_t r) {
            const float *A = Lxyz + 3 * (size_t)p, *B = Lxyz + 3 * (size_t)q, *C = Lxyz + 3 * (size_t)r;
            // collinear iff the cross product vanishes exactly: use orient with
            // the three axis-offset points
            for (int ax = 0; ax < 3; ++ax) {
                float D[3] = {A[0], A[1], A[2]};
                D[ax] += 1.0f;
                if (D[ax] == A[ax]) D[ax] = A[ax] * 2.0f + 1.0f;
                if (tr.pr.orient(A, B, C, D) != 0) return false;
            }
            return true;
        };
        for (size_t i = ia1 + 1; i < seq.size(); ++i)
            if (!collinear(a0, a1, seq[i])) { a2 = seq[i]; ia2 = i; break; }
        if (a2 < 0) {
            set_error("flood_delaunay: all landmarks are collinear");
            return FLOOD_EDEGENERATE;
        }
        for (size_t i = 1; i < seq.size(); ++i) {
            if (i == ia1 || i == ia2) continue;
            if (tr.pr.orient(Lxyz + 3 * (size_t)a0, Lxyz + 3 * (size_t)a1, Lxyz + 3 * (size_t)a2, Lxyz + 3 * (size_t)seq[i]) != 0) {
                a3 = seq[i];
                ia3 = i;
                break;
            }
        }
        if (a3 < 0) {
            set_error("flood_delaunay: all landmarks are coplanar");
            return FLOOD_EDEGENERATE;
        }
        if (tr.pr.orient(Lxyz + 3 * (size_t)a0, Lxyz + 3 * (size_t)a1, Lxyz + 3 * (size_t)a2, Lxyz + 3 * (size_t)a3) < 0)
            std::swap(a0, a1);
        // tet 0 finite, tets 1..4 infinite (facet i of tet 0, two vertices swapped)
        tr.t.resize(5);
        tr.dead.assign(5, 0);
        tr.in_cav.assign(5, 0);
        tr.tested.assign(5, 0);
        Tet &t0 = tr.t[0];
        int vs[4] = {a0, a1, a2, a3};
        for (int i = 0; i < 4; ++i) {
            t0.v[i] = vs[i];
            t0.n[i] = 1 + i;
        }
        for (int i = 0; i < 4; ++i) {
            Tet x;
            for (int k = 0; k < 4; ++k) x.v[k] = vs[k];
            x.v[i] = INF;
            // swap two finite slots to flip the parity
            int s0 = -1, s1 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != i) { if (s0 < 0) s0 = k; else if (s1 < 0) s1 = k; }
            std::swap(x.v[s0], x.v[s1]);
            // neighbours: across the INF slot -> tet 0; across a finite slot ->
            // the infinite tet built on the facet without that vertex
            for (int k = 0; k < 4; ++k) {
                if (k == i) {
                    x.n[k] = 0;
                } else {
                    int vk = x.v[k];
                    int fi = 0;
                    for (int m = 0; m < 4; ++m)
                        if (vs[m] == vk) fi = m;
                    x.n[k] = 1 + fi;
                }
            }
            tr.t[1 + i] = x;
        }
        tr.last = 0;
        for (size_t i = 0; i < seq.size(); ++i) {
            if (i == 0 || i == ia1 || i == ia2 || i == ia3) continue;
            tr.insert(seq[i]);
        }
        // extract
        flood_complex *cx = new flood_complex();
        cx->L = L;
        cx->fallbacks = tr.pr.fallbacks;
        for (size_t i = 0; i < tr.t.size(); ++i) {
            if (tr.dead[i] || tr.infinite((int)i)) continue;
            std::array<int32_t, 4> r = {tr.t[i].v[0], tr.t[i].v[1], tr.t[i].v[2], tr.t[i].v[3]};
            std::sort(r.begin(), r.end());
            cx->T.push_back(r);
        }
        std::sort(cx->T.begin(), cx->T.end());
        // faces: every facet of every tet as a record (sorted vertices, owner
        // row, slot); a counting sort by the first vertex and a sort of each
        // small bucket by the others put equal facets next to each other in
        // lexicographic order, so a facet's rank is its row, written straight
        // into the owner's facet map (facet i omits vertex i)
        struct Rec {
            int32_t a, b, c, row, slot;
        };
        std::vector<Rec> rec, grouped;
        std::vector<int64_t> start(L + 1);
        auto group = [&]() {
            std::fill(start.begin(), start.end(), 0);
            for (const Rec &r : rec) ++start[r.a + 1];
            for (int32_t v = 0; v < L; ++v) start[v + 1] += start[v];
            grouped.resize(rec.size());
            std::vector<int64_t> cur(start.begin(), start.end() - 1);
            for (const Rec &r : rec) grouped[cur[r.a]++] = r;
            for (int32_t v = 0; v < L; ++v)
                std::sort(grouped.begin() + start[v], grouped.begin() + start[v + 1], [](const Rec &x, const Rec &y) {
                    return x.b != y.b ? x.b < y.b : x.c < y.c;
                });
        };
        rec.reserve(cx->T.size() * 4);
        for (size_t j = 0; j < cx->T.size(); ++j) {
            const auto &r = cx->T[j];
            rec.push_back(Rec{r[1], r[2], r[3], (int32_t)j, 0});
            rec.push_back(Rec{r[0], r[2], r[3], (int32_t)j, 1});
            rec.push_back(Rec{r[0], r[1], r[3], (int32_t)j, 2});
            rec.push_back(Rec{r[0], r[1], r[2], (int32_t)j, 3});
        }
        group();
        cx->tet_tris.resize(cx->T.size());
        cx->F.reserve(grouped.size() / 2 + 8);
        for (size_t i = 0; i < grouped.size(); ++i) {
            const Rec &r = grouped[i];
            if (i == 0 || r.a != grouped[i - 1].a || r.b != grouped[i - 1].b || r.c != grouped[i - 1].c)
                cx->F.push_back({r.a, r.b, r.c});
            cx->tet_tris[r.row][r.slot] = (int32_t)cx->F.size() - 1;
        }
        rec.clear();
        rec.reserve(cx->F.size() * 3);
        for (size_t j = 0; j < cx->F.size(); ++j) {
            const auto &f = cx->F[j];
            rec.push_back(Rec{f[1], f[2], 0, (int32_t)j, 0});
            rec.push_back(Rec{f[0], f[2], 0, (int32_t)j, 1});
            rec.push_back(Rec{f[0], f[1], 0, (int32_t)j, 2});
        }
        group();
        cx->tri_edges.resize(cx->F.size());
        cx->E.reserve(grouped.size() / 3 + 8);
        for (size_t i = 0; i < grouped.size(); ++i) {
            const Rec &r = grouped[i];
            if (i == 0 || r.a != grouped[i - 1].a || r.b != grouped[i - 1].b) cx->E.push_back({r.a, r.b});
            cx->tri_edges[r.row][r.slot] = (int32_t)cx->E.size() - 1;
        }
        int64_t euler = (int64_t)L - (int64_t)cx->E.size() + (int64_t)cx->F.size() - (int64_t)cx->T.size();
        std::vector<char> used(L, 0);
        for (auto &r : cx->T)
            for (int k = 0; k < 4; ++k) used[r[k]] = 1;
        bool all_used = std::all_of(used.begin(), used.end(), [](char c) { return c != 0; });
        if (euler != 1 || !all_used) {
            delete cx;
            set_error("flood_delaunay: internal consistency check failed (Euler characteristic or unused landmark)");
            return FLOOD_EDEGENERATE;
        }
        *out = cx;
        return FLOOD_OK;
    } catch (Degenerate &) {
        set_error("flood_delaunay: exactly degenerate configuration (coplanar or cospherical points)");
        return FLOOD_EDEGENERATE;
    } catch (std::bad_alloc &) {
        set_error("flood_delaunay: out of host memory");
        return FLOOD_ENOMEM;
    }
}

extern "C" flood_status flood_complex_counts(const flood_complex *cx, int64_t counts[5]) {
    if (!cx || !counts) {
        flood_host::set_error("flood_complex_counts: NULL argument");
        return FLOOD_EINVAL;
    }
    counts[0] = cx->L;
    counts[1] = (int64_t)cx->E.size();
    counts[2] = (int64_t)cx->F.size();
    counts[3] = (int64_t)cx->T.size();
    counts[4] = cx->fallbacks;
    return FLOOD_OK;
}

extern "C" flood_status flood_complex_export(const flood_complex *cx, int32_t *edges, int32_t *tris, int32_t *tets,
                                             int32_t *tri_edges, int32_t *tet_tris) {
    if (!cx) {
        flood_host::set_error("flood_complex_export: NULL complex");
        return FLOOD_EINVAL;
    }
    // (an empty array, such as the tetrahedra of a planar complex, copies
    // nothing: memcpy is not called with its possibly null data pointer)
    auto put = [](int32_t *dst, const auto &v) {
        if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    put(edges, cx->E);
    put(tris, cx->F);
    put(tets, cx->T);
    put(tri_edges, cx->tri_edges);
    put(tet_tris, cx->tet_tris);
    return FLOOD_OK;
}

extern "C" void flood_complex_free(flood_complex *cx) { delete cx; }

// ---------------------------------------------------------------------------
// Delaunay triangulation in the plane (ambient dimension 2): the same
// incremental construction with triangles, the orientation predicate
// orient2(a,b,c) = det[a-c; b-c] and the in-circle predicate
// incircle(a,b,c,d) = det of the rows (p - d, |p - d|^2), p in (a,b,c), which
// is positive iff d lies strictly inside the circle through a positively
// oriented (a,b,c).  FP64 filter, exact integer fallback.

namespace {

int orient2_exact(const float *a, const float *b, const float *c) {
    const float A[3] = {a[0], a[1], 0.f}, B[3] = {b[0], b[1], 0.f}, C[3] = {c[0], c[1], 0.f};
    const float *p[3] = {A, B, C};
    ExactCoords x = exact_scale(p, 3);
    Big u0 = x.c[0][0] - x.c[2][0], u1 = x.c[0][1] - x.c[2][1];
    Big w0 = x.c[1][0] - x.c[2][0], w1 = x.c[1][1] - x.c[2][1];
    return (u0 * w1 - u1 * w0).sign;
}

int incircle_exact(const float *a, const float *b, const float *c, const float *d) {
    const float A[3] = {a[0], a[1], 0.f}, B[3] = {b[0], b[1], 0.f}, C[3] = {c[0], c[1], 0.f}, D[3] = {d[0], d[1], 0.f};
    const float *p[4] = {A, B, C, D};
    ExactCoords x = exact_scale(p, 4);
    Big R[3][3];
    for (int i = 0; i < 3; ++i) {
        R[i][0] = x.c[i][0] - x.c[3][0];
        R[i][1] = x.c[i][1] - x.c[3][1];
        R[i][2] = R[i][0] * R[i][0] + R[i][1] * R[i][1];
    }
    return det3(R[0], R[1], R[2]).sign;
}

struct Predicates2 {
    int64_t fallbacks = 0;
    int orient(const float *a, const float *b, const float *c) {
        const double ax = (double)a[0] - c[0], ay = (double)a[1] - c[1];
        const double bx = (double)b[0] - c[0], by = (double)b[1] - c[1];
        const double det = ax * by - ay * bx;
        const double perm = std::fabs(ax * by) + std::fabs(ay * bx);
        if (std::fabs(det) > 1e-13 * perm) return det > 0 ? 1 : -1;
        ++fallbacks;
        return orient2_exact(a, b, c);
    }
    int incircle(const float *a, const float *b, const float *c, const float *d) {
        const float *p[3] = {a, b, c};
        double R[3][3];
        for (int i = 0; i < 3; ++i) {
            R[i][0] = (double)p[i][0] - d[0];
            R[i][1] = (double)p[i][1] - d[1];
            R[i][2] = R[i][0] * R[i][0] + R[i][1] * R[i][1];
        }
        const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                           R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                           R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
        const double perm = std::fabs(R[0][0]) * (std::fabs(R[1][1] * R[2][2]) + std::fabs(R[1][2] * R[2][1])) +
                            std::fabs(R[0][1]) * (std::fabs(R[1][0] * R[2][2]) + std::fabs(R[1][2] * R[2][0])) +
                            std::fabs(R[0][2]) * (std::fabs(R[1][0] * R[2][1]) + std::fabs(R[1][1] * R[2][0]));
        if (std::fabs(det) > 1e-12 * perm) return det > 0 ? 1 : -1;
        ++fallbacks;
        return incircle_exact(a, b, c, d);
    }
};

struct Tri {
    int v[3];
    int n[3];  // neighbour across the edge opposite v[i]
};

// triangles with an infinite vertex (-1) outside the hull; every triangle
// positively oriented (for an infinite one: replacing the infinite vertex by a
// point q gives a positive orientation iff q lies strictly beyond its hull edge)
struct Triangulation2 {
    const float *P;  // [L][2]
    Predicates2 pr;
    std::vector<Tri> t;
    std::vector<char> dead;
    std::vector<uint32_t> in_cav, tested;
    std::vector<int> free_list, cavity, stack;
    struct VertSlot {
        int v, tri, edge;
    };
    std::vector<VertSlot> open_v;
    uint32_t ins = 0;
    int last = 0;
    uint64_t rng = 0x2545f4914f6cdd1dull;

    const float *pt(int i) const { return P + 2 * (size_t)i; }
    static bool infinite_v(const Tri &x) { return x.v[0] == INF || x.v[1] == INF || x.v[2] == INF; }
    bool infinite(int ti) const { return infinite_v(t[ti]); }
    int new_tri() {
        int i;
        if (!free_list.empty()) {
            i = free_list.back();
            free_list.pop_back();
        } else {
            t.push_back(Tri{});
            dead.push_back(0);
            in_cav.push_back(0);
            tested.push_back(0);
            i = (int)t.size() - 1;
        }
        dead[i] = 0;
        in_cav[i] = 0;
        tested[i] = 0;
        return i;
    }
    uint32_t rnd() {
        rng ^= rng << 13;
        rng ^= rng >> 7;
        rng ^= rng << 17;
        return (uint32_t)rng;
    }
    int orient_with(int ti, int i, int q) {
        const Tri &x = t[ti];
        const float *p[3];
        for (int k = 0; k < 3; ++k) p[k] = (k == i) ? pt(q) : pt(x.v[k]);
        return pr.orient(p[0], p[1], p[2]);
    }
    bool conflict(int ti, int q) {
        const Tri &x = t[ti];
        for (int k = 0; k < 3; ++k)
            if (x.v[k] == INF) {
                int o = orient_with(ti, k, q);
                if (o == 0) throw Degenerate();
                return o > 0;
            }
        int s = pr.incircle(pt(x.v[0]), pt(x.v[1]), pt(x.v[2]), pt(q));
        if (s == 0) throw Degenerate();
        return s > 0;
    }
    int locate(int q) {
        int cur = last;
        size_t steps = 0, limit = 8 * t.size() + 64;
        while (steps++ < limit) {
            if (infinite(cur)) return cur;
            int start = (int)(rnd() % 3u);
            int moved = -1;
            for (int r = 0; r < 3; ++r) {
                int i = (start + r) % 3;
                if (orient_with(cur, i, q) < 0) {
                    moved = t[cur].n[i];
                    break;
                }
            }
            if (moved < 0) return cur;
            cur = moved;
        }
        for (int i = 0; i < (int)t.size(); ++i)
            if (!dead[i] && conflict(i, q)) return i;
        throw Degenerate();
    }
    void insert(int q) {
        int c0 = locate(q);
        if (!conflict(c0, q)) throw Degenerate();
        ++ins;
        cavity.clear();
        stack.clear();
        stack.push_back(c0);
        in_cav[c0] = ins;
        tested[c0] = ins;
        while (!stack.empty()) {
            int c = stack.back();
            stack.pop_back();
            cavity.push_back(c);
            for (int i = 0; i < 3; ++i) {
                int nb = t[c].n[i];
                if (tested[nb] == ins) continue;
                tested[nb] = ins;
                if (conflict(nb, q)) {
                    in_cav[nb] = ins;
                    stack.push_back(nb);
                }
            }
        }
        // new triangles on the cavity boundary; the edges through q are glued
        // by their other vertex (each boundary vertex meets two new triangles)
        open_v.clear();
        int created_finite = -1;
        for (int c : cavity) {
            for (int i = 0; i < 3; ++i) {
                int nb = t[c].n[i];
                if (in_cav[nb] == ins) continue;
                Tri x = t[c];
                x.v[i] = q;
                for (int k = 0; k < 3; ++k) x.n[k] = -1;
                x.n[i] = nb;
                if (!infinite_v(x) && pr.orient(pt(x.v[0]), pt(x.v[1]), pt(x.v[2])) <= 0) throw Degenerate();
                int nt = new_tri();
                t[nt] = x;
                for (int k = 0; k < 3; ++k)
                    if (t[nb].n[k] == c) t[nb].n[k] = nt;
                if (created_finite < 0 && !infinite_v(x)) created_finite = nt;
                // the edge opposite slot j (j != i) joins q and the vertex in
                // the third slot
                for (int j = 0; j < 3; ++j) {
                    if (j == i) continue;
                    const int other = x.v[3 - i - j];
                    size_t at = 0;
                    while (at < open_v.size() && open_v[at].v != other) ++at;
                    if (at == open_v.size()) {
                        open_v.push_back(VertSlot{other, nt, j});
                    } else {
                        t[nt].n[j] = open_v[at].tri;
                        t[open_v[at].tri].n[open_v[at].edge] = nt;
                        open_v[at] = open_v.back();
                        open_v.pop_back();
                    }
                }
            }
        }
        if (!open_v.empty()) throw Degenerate();
        for (int c : cavity) {
            dead[c] = 1;
            free_list.push_back(c);
        }
        if (created_finite >= 0) last = created_finite;
    }
};

}  // namespace

extern "C" flood_status flood_delaunay2d(const float *Lxy, int32_t L, flood_complex **out) {
    using flood_host::set_error;
    if (!out) {
        set_error("flood_delaunay2d: out is NULL");
        return FLOOD_EINVAL;
    }
    *out = nullptr;
    if (!Lxy || L < 0) {
        set_error("flood_delaunay2d: bad arguments");
        return FLOOD_EINVAL;
    }
    if (L < 3) {
        set_error("flood_delaunay2d: need at least 3 landmarks");
        return FLOOD_EDEGENERATE;
    }
    for (int64_t i = 0; i < 2 * (int64_t)L; ++i)
        if (!std::isfinite(Lxy[i])) {
            set_error("flood_delaunay2d: non-finite coordinate");
            return FLOOD_EINVAL;
        }
    try {
        std::vector<int32_t> ord(L);
        for (int32_t i = 0; i < L; ++i) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            return std::lexicographical_compare(Lxy + 2 * (size_t)a, Lxy + 2 * (size_t)a + 2, Lxy + 2 * (size_t)b,
                                                Lxy + 2 * (size_t)b + 2);
        });
        for (int32_t i = 1; i < L; ++i)
            if (std::memcmp(Lxy + 2 * (size_t)ord[i], Lxy + 2 * (size_t)ord[i - 1], 2 * sizeof(float)) == 0) {
                set_error("flood_delaunay2d: duplicate landmark coordinates");
                return FLOOD_EDEGENERATE;
            }
        // Morton insertion order
        float lo[2] = {Lxy[0], Lxy[1]}, hi[2] = {Lxy[0], Lxy[1]};
        for (int32_t i = 0; i < L; ++i)
            for (int a = 0; a < 2; ++a) {
                lo[a] = std::min(lo[a], Lxy[2 * (size_t)i + a]);
                hi[a] = std::max(hi[a], Lxy[2 * (size_t)i + a]);
            }
        std::vector<std::pair<uint64_t, int32_t>> mk(L);
        for (int32_t i = 0; i < L; ++i) {
            uint64_t code = 0;
            for (int a = 0; a < 2; ++a) {
                double ext = (double)hi[a] - lo[a];
                double u = ext > 0 ? ((double)Lxy[2 * (size_t)i + a] - lo[a]) / ext : 0.0;
                uint64_t qv = (uint64_t)std::min(4294967295.0, std::max(0.0, u * 4294967295.0));
                for (int bit = 0; bit < 32; ++bit) code |= ((qv >> bit) & 1ull) << (2 * bit + a);
            }
            mk[i] = {code, i};
        }
        std::sort(mk.begin(), mk.end());
        Triangulation2 tr;
        tr.P = Lxy;
        std::vector<int32_t> seq(L);
        for (int32_t i = 0; i < L; ++i) seq[i] = mk[i].second;
        // first triangle: three points in insertion order that are not collinear
        int32_t a0 = seq[0], a1 = seq[1], a2 = -1;
        size_t ia2 = 0;
        for (size_t i = 2; i < seq.size(); ++i)
            if (tr.pr.orient(Lxy + 2 * (size_t)a0, Lxy + 2 * (size_t)a1, Lxy + 2 * (size_t)seq[i]) != 0) {
                a2 = seq[i];
                ia2 = i;
                break;
            }
        if (a2 < 0) {
            set_error("flood_delaunay2d: all landmarks are collinear");
            return FLOOD_EDEGENERATE;
        }
        if (tr.pr.orient(Lxy + 2 * (size_t)a0, Lxy + 2 * (size_t)a1, Lxy + 2 * (size_t)a2) < 0) std::swap(a0, a1);
        // triangle 0 finite; triangles 1..3 infinite, triangle 1 + i on the hull
        // edge opposite vertex i of triangle 0 (its two vertices swapped)
        tr.t.resize(4);
        tr.dead.assign(4, 0);
        tr.in_cav.assign(4, 0);
        tr.tested.assign(4, 0);
        const int vs[3] = {a0, a1, a2};
        for (int i = 0; i < 3; ++i) {
            tr.t[0].v[i] = vs[i];
            tr.t[0].n[i] = 1 + i;
        }
        for (int i = 0; i < 3; ++i) {
            // edge opposite vertex i: (vs[i+1], vs[i+2]) in the triangle's
            // order; the infinite triangle takes it reversed
            const int p = vs[(i + 1) % 3], q = vs[(i + 2) % 3];
            Tri x;
            x.v[0] = INF;
            x.v[1] = q;
            x.v[2] = p;
            x.n[0] = 0;  // across the finite edge
            // across the edge opposite q (INF, p): the infinite triangle on the
            // hull edge that contains p and the third vertex, i.e. opposite q
            int iq = 0, ip = 0;
            for (int m = 0; m < 3; ++m) {
                if (vs[m] == q) iq = m;
                if (vs[m] == p) ip = m;
            }
            x.n[1] = 1 + iq;
            x.n[2] = 1 + ip;
            tr.t[1 + i] = x;
        }
        tr.last = 0;
        for (size_t i = 0; i < seq.size(); ++i) {
            if (i == 0 || i == 1 || i == ia2) continue;
            tr.insert(seq[i]);
        }
        flood_complex *cx = new flood_complex();
        cx->L = L;
        cx->fallbacks = tr.pr.fallbacks;
        for (size_t i = 0; i < tr.t.size(); ++i) {
            if (tr.dead[i] || tr.infinite((int)i)) continue;
            std::array<int32_t, 3> r = {tr.t[i].v[0], tr.t[i].v[1], tr.t[i].v[2]};
            std::sort(r.begin(), r.end());
            cx->F.push_back(r);
        }
        std::sort(cx->F.begin(), cx->F.end());
        std::vector<std::array<int32_t, 4>> rec;  // (a, b, triangle row, slot)
        rec.reserve(cx->F.size() * 3);
        for (size_t j = 0; j < cx->F.size(); ++j) {
            const auto &f = cx->F[j];
            rec.push_back({f[1], f[2], (int32_t)j, 0});
            rec.push_back({f[0], f[2], (int32_t)j, 1});
            rec.push_back({f[0], f[1], (int32_t)j, 2});
        }
        std::sort(rec.begin(), rec.end());
        cx->tri_edges.resize(cx->F.size());
        for (size_t i = 0; i < rec.size(); ++i) {
            if (i == 0 || rec[i][0] != rec[i - 1][0] || rec[i][1] != rec[i - 1][1]) cx->E.push_back({rec[i][0], rec[i][1]});
            cx->tri_edges[rec[i][2]][rec[i][3]] = (int32_t)cx->E.size() - 1;
        }
        const int64_t euler = (int64_t)L - (int64_t)cx->E.size() + (int64_t)cx->F.size();
        std::vector<char> used(L, 0);
        for (auto &r : cx->F)
            for (int k = 0; k < 3; ++k) used[r[k]] = 1;
        const bool all_used = std::all_of(used.begin(), used.end(), [](char c) { return c != 0; });
        if (euler != 1 || !all_used) {
            delete cx;
            set_error("flood_delaunay2d: internal consistency check failed (Euler characteristic or unused landmark)");
            return FLOOD_EDEGENERATE;
        }
        *out = cx;
        return FLOOD_OK;
    } catch (Degenerate &) {
        set_error("flood_delaunay2d: exactly degenerate configuration (collinear or cocircular points)");
        return FLOOD_EDEGENERATE;
    } catch (std::bad_alloc &) {
        set_error("flood_delaunay2d: out of host memory");
        return FLOOD_ENOMEM;
    }
}
