// Persistence diagrams of a flood filtration over Z/2 (host).
//
// The flood values make the Delaunay complex a filtered complex (Sec. 2:
// sublevel complexes f^{-1}((-inf, t]); the monotone closure of Sec. 4.1
// guarantees f(face) <= f(coface)), and the homology step that follows the
// flooding computes its persistence diagrams in dimensions 0..2 (the paper
// uses Gudhi for it).  Simplices are totally ordered by (f, dimension,
// vertex tuple); the boundary matrix is reduced column by column, dimension
// by dimension from the top, and a column that became a pivot row is
// skipped when its own dimension comes (the clearing shortcut).  Columns
// are kept as sorted vectors of filtration positions and added by merging.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "../../include/flood.h"

namespace flood_host {
void set_error(const std::string &msg);
}

struct flood_diagram {
    // per dimension p = 0..2: (birth, death) values and the simplex rows
    std::vector<float> birth[3], death[3];
    std::vector<int64_t> birth_row[3], death_row[3];
};

namespace {

using Col = std::vector<int32_t>;

// a ^ b for sorted columns
void add_into(Col &a, const Col &b, Col &tmp) {
    tmp.clear();
    size_t i = 0, j = 0;
    while (i < a.size() && j < b.size()) {
        if (a[i] < b[j]) tmp.push_back(a[i++]);
        else if (b[j] < a[i]) tmp.push_back(b[j++]);
        else {
            ++i;
            ++j;
        }
    }
    while (i < a.size()) tmp.push_back(a[i++]);
    while (j < b.size()) tmp.push_back(b[j++]);
    a.swap(tmp);
}

}  // namespace

extern "C" flood_status flood_persistence(const int64_t n[4], const int32_t *edges, const int32_t *tri_edges,
                                          const int32_t *tet_tris, const float *const f[4], flood_diagram **out) {
    using flood_host::set_error;
    if (!out) {
        set_error("flood_persistence: out is NULL");
        return FLOOD_EINVAL;
    }
    *out = nullptr;
    if (!n || !f) {
        set_error("flood_persistence: NULL argument");
        return FLOOD_EINVAL;
    }
    for (int d = 0; d < 4; ++d)
        if (n[d] < 0 || (n[d] > 0 && !f[d])) {
            set_error("flood_persistence: negative count or missing f");
            return FLOOD_EINVAL;
        }
    if ((n[1] && !edges) || (n[2] && !tri_edges) || (n[3] && !tet_tris)) {
        set_error("flood_persistence: missing simplex rows or face maps");
        return FLOOD_EINVAL;
    }
    const int64_t total = n[0] + n[1] + n[2] + n[3];
    if (total >= (int64_t)std::numeric_limits<int32_t>::max()) {
        set_error("flood_persistence: more than 2^31 - 1 simplices");
        return FLOOD_EUNSUPPORTED;
    }
    const int64_t base[5] = {0, n[0], n[0] + n[1], n[0] + n[1] + n[2], total};
    // facets of simplex (d, row) as global ids; checks ids and monotonicity
    auto facets = [&](int d, int64_t r, int64_t *g) -> int {
        if (d == 1) {
            g[0] = edges[2 * r];
            g[1] = edges[2 * r + 1];
            return 2;
        }
        const int32_t *m = d == 2 ? tri_edges + 3 * r : tet_tris + 4 * r;
        for (int i = 0; i <= d; ++i) g[i] = base[d - 1] + m[i];
        return d + 1;
    };
    std::vector<float> val((size_t)total);
    for (int d = 0; d < 4; ++d)
        for (int64_t r = 0; r < n[d]; ++r) {
            const float v = f[d][r];
            if (std::isnan(v)) {
                set_error("flood_persistence: NaN filtration value");
                return FLOOD_EINVAL;
            }
            val[(size_t)(base[d] + r)] = v;
        }
    for (int d = 1; d < 4; ++d)
        for (int64_t r = 0; r < n[d]; ++r) {
            int64_t g[4];
            const int k = facets(d, r, g);
            for (int i = 0; i < k; ++i) {
                const int64_t id = g[i] - base[d - 1];  // row of the facet in dimension d-1
                if (id < 0 || id >= n[d - 1]) {
                    set_error("flood_persistence: face index out of range");
                    return FLOOD_EINVAL;
                }
                if (val[(size_t)g[i]] > val[(size_t)(base[d] + r)]) {
                    set_error("flood_persistence: f(face) > f(coface): not a filtration");
                    return FLOOD_EINVAL;
                }
            }
        }
    flood_diagram *dg = new (std::nothrow) flood_diagram();
    if (!dg) {
        set_error("flood_persistence: out of host memory");
        return FLOOD_ENOMEM;
    }
    try {
        // filtration order: (f, dimension, row); global ids already run in
        // (dimension, row) order, so ties in f fall back to the id
        std::vector<int32_t> order((size_t)total);
        for (int64_t g = 0; g < total; ++g) order[(size_t)g] = (int32_t)g;
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return val[(size_t)a] < val[(size_t)b] || (val[(size_t)a] == val[(size_t)b] && a < b);
        });
        std::vector<int32_t> pos((size_t)total);
        for (int64_t i = 0; i < total; ++i) pos[(size_t)order[(size_t)i]] = (int32_t)i;
        auto dim_of = [&](int64_t g) { return g < base[1] ? 0 : (g < base[2] ? 1 : (g < base[3] ? 2 : 3)); };

        std::vector<int32_t> pivot_col((size_t)total, -1);  // position of the column whose low is this row
        std::vector<uint8_t> cleared((size_t)total, 0), zero((size_t)total, 0);
        std::vector<Col> reduced((size_t)total);
        Col col, tmp;
        for (int d = 3; d >= 1; --d) {
            for (int64_t i = 0; i < total; ++i) {
                const int64_t g = order[(size_t)i];
                if (dim_of(g) != d || cleared[(size_t)i]) continue;
                int64_t fg[4];
                const int k = facets(d, g - base[d], fg);
                col.clear();
                for (int t = 0; t < k; ++t) col.push_back(pos[(size_t)fg[t]]);
                std::sort(col.begin(), col.end());
                while (!col.empty()) {
                    const int32_t low = col.back();
                    const int32_t p = pivot_col[(size_t)low];
                    if (p < 0) break;
                    add_into(col, reduced[(size_t)p], tmp);
                }
                if (col.empty()) {
                    zero[(size_t)i] = 1;
                } else {
                    const int32_t low = col.back();
                    pivot_col[(size_t)low] = (int32_t)i;
                    cleared[(size_t)low] = 1;
                    reduced[(size_t)i] = col;
                }
            }
        }
        // pairs (birth position = low, death position = column), positive
        // persistence only, in the filtration order of the birth simplex;
        // then the essential classes (unpaired positive simplices)
        for (int64_t i = 0; i < total; ++i) {
            const int64_t g = order[(size_t)i];
            const int p = dim_of(g);
            if (p > 2) continue;
            const int32_t j = pivot_col[(size_t)i];
            if (j >= 0) {
                const int64_t gd = order[(size_t)j];
                if (val[(size_t)gd] > val[(size_t)g]) {
                    dg->birth[p].push_back(val[(size_t)g]);
                    dg->death[p].push_back(val[(size_t)gd]);
                    dg->birth_row[p].push_back(g - base[p]);
                    dg->death_row[p].push_back(gd - base[p + 1]);
                }
            }
        }
        for (int64_t i = 0; i < total; ++i) {
            const int64_t g = order[(size_t)i];
            const int p = dim_of(g);
            if (p > 2 || cleared[(size_t)i] || pivot_col[(size_t)i] >= 0) continue;
            if (p > 0 && !zero[(size_t)i]) continue;  // a negative simplex
            dg->birth[p].push_back(val[(size_t)g]);
            dg->death[p].push_back(std::numeric_limits<float>::infinity());
            dg->birth_row[p].push_back(g - base[p]);
            dg->death_row[p].push_back(-1);
        }
    } catch (const std::bad_alloc &) {
        delete dg;
        set_error("flood_persistence: out of host memory");
        return FLOOD_ENOMEM;
    }
    *out = dg;
    return FLOOD_OK;
}

extern "C" flood_status flood_diagram_counts(const flood_diagram *dg, int64_t counts[3]) {
    if (!dg || !counts) {
        flood_host::set_error("flood_diagram_counts: NULL argument");
        return FLOOD_EINVAL;
    }
    for (int p = 0; p < 3; ++p) counts[p] = (int64_t)dg->birth[p].size();
    return FLOOD_OK;
}

extern "C" flood_status flood_diagram_export(const flood_diagram *dg, int32_t dim, float *birth, float *death,
                                             int64_t *birth_row, int64_t *death_row) {
    if (!dg || dim < 0 || dim > 2) {
        flood_host::set_error("flood_diagram_export: NULL handle or dim outside [0, 2]");
        return FLOOD_EINVAL;
    }
    if (birth) std::copy(dg->birth[dim].begin(), dg->birth[dim].end(), birth);
    if (death) std::copy(dg->death[dim].begin(), dg->death[dim].end(), death);
    if (birth_row) std::copy(dg->birth_row[dim].begin(), dg->birth_row[dim].end(), birth_row);
    if (death_row) std::copy(dg->death_row[dim].begin(), dg->death_row[dim].end(), death_row);
    return FLOOD_OK;
}

extern "C" void flood_diagram_free(flood_diagram *dg) { delete dg; }
