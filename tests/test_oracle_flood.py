"""Pins for the oracle's sampled flood values f_P (FP64)."""
import os
from math import comb

import numpy as np
import pytest

import synth
from oracle import delaunay as D
from oracle import flood as FL
from oracle import fps as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _complex(L):
    T = D.qhull_tets(L)
    D.certify(L, T)
    E, Fc, te, tt = D.faces(T)
    return dict(E=E, F=Fc, T=T, tri_edges=te, tet_tris=tt, L=len(L))


def _small_problem(seed=0, n=400, nl=16):
    X = synth.config_cloud(1, n_points=n) if seed == 0 else \
        np.random.default_rng(seed).random((n, 3)).astype(np.float32)
    idx, _ = F.fps(X, nl)
    L = X[idx]
    return X, L, _complex(L)


def test_sample_grid_sizes_golden():
    # Lemma 6 grid: C(k+d, d) points; the paper quotes 210 / 1540 at 20 points per edge
    for line in open(os.path.join(GOLDEN, "sample_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        d, k, cnt = map(int, line.split())
        assert len(FL.samples(d, k)) == cnt
    for d in range(4):
        for k in range(1, 12):
            S = FL.samples(d, k)
            assert len(S) == comb(k + d, d)
            assert np.all(S.sum(1) == k) and np.all(S >= 0)
            assert len(np.unique(S, axis=0)) == len(S)
            # lexicographically descending
            keys = [tuple(r) for r in S]
            assert keys == sorted(keys, reverse=True)


def test_vertices_zero_and_bounds():
    X, L, cx = _small_problem()
    k = 4
    vals = FL.flood_all(X, L, cx, k)
    assert np.all(vals[0][0] == 0.0)        # L inside X: vertices flooded at r = 0
    E = cx["E"]
    half = np.sqrt(((L[E[:, 0]].astype(float) - L[E[:, 1]]) ** 2).sum(1)) / 2
    assert np.all(vals[1][0] <= half * (1 + 1e-12))
    # per-sample vertex bound (proof of Lemma 7): f <= max_p min_i |p - v_i|
    for d, key in ((1, "E"), (2, "F"), (3, "T")):
        S = FL.samples(d, k) / k
        V = L[cx[key]].astype(np.float64)
        P = np.einsum("sd,ndc->nsc", S, V)
        ub = np.sqrt(((P[:, :, None, :] - V[:, None, :, :]) ** 2).sum(-1)).min(-1).max(-1)
        assert np.all(vals[d][0] <= ub * (1 + 1e-12))


def test_brute_equals_masked():
    # Lemma 7: the enclosing-ball mask loses nothing when L is inside X
    X, L, cx = _small_problem(seed=3, n=3000, nl=40)
    for k in (2, 5):
        b = FL.flood_all(X, L, cx, k, "brute")
        m = FL.flood_all(X, L, cx, k, "masked")
        for d in range(4):
            for i in range(3):
                assert np.array_equal(b[d][i], m[d][i])


def test_closure_is_noop_on_nested_grid():
    X, L, cx = _small_problem()
    vals = FL.flood_all(X, L, cx, 6)
    FL.assert_closure_noop(vals, cx)
    c = FL.closure(vals, cx)
    # monotone: f(face) <= f(coface)
    assert np.all(c[1][cx["tri_edges"]] <= c[2][:, None])
    assert np.all(c[2][cx["tet_tris"]] <= c[3][:, None])


def test_winners_attain_value():
    X, L, cx = _small_problem()
    k = 4
    vals = FL.flood_all(X, L, cx, k)
    for d, key in ((1, "E"), (2, "F"), (3, "T")):
        f, wa, wx = vals[d]
        assert np.all(wa[:, : d + 1].sum(1) == k)
        sp = FL.winner_points(L, cx[key], wa, k)
        dd = np.sqrt(((sp - X[wx].astype(np.float64)) ** 2).sum(1))
        assert np.array_equal(dd, f)
        # x* is a nearest point of s*
        dall = np.sqrt(((sp[:, None, :] - X[None].astype(np.float64)) ** 2).sum(-1)).min(1)
        assert np.array_equal(dall, f)


@pytest.mark.parametrize("seed", range(5))
def test_sandwich_with_exact_radius(seed):
    # Thm 5 + Lemma 6: 0 <= r_exact - f_P <= h(sigma) = sqrt(sum |vi-vj|^2)/k
    rng = np.random.default_rng(seed)
    X = rng.random((14, 3))
    for d in (1, 2, 3):
        V = X[rng.choice(14, d + 1, replace=False)]
        r, cnt = FL.r_exact(X, V)
        assert cnt > 0
        simp = np.arange(d + 1).reshape(1, -1)
        for k in (2, 3, 5):
            f, _, _ = FL.flood_dim(X, V, simp, d, k)
            h = FL.h_grid(V, simp, k)[0]
            assert -1e-12 <= r - f[0] <= h + 1e-12, (d, k, r, f[0], h)
        # a fine grid pins r_exact itself from below and above
        f, _, _ = FL.flood_dim(X, V, simp, d, 60)
        assert f[0] <= r + 1e-12 and r - f[0] <= FL.h_grid(V, simp, 60)[0] + 1e-12


def test_sandwich_landmarks_not_in_x():
    # Def. 1 does not need L inside X; brute mode handles it
    rng = np.random.default_rng(11)
    X = rng.random((12, 3))
    V = rng.random((4, 3))
    r, _ = FL.r_exact(X, V)
    f, _, _ = FL.flood_dim(X, V, np.arange(4).reshape(1, -1), 3, 4)
    assert 0 <= r - f[0] <= FL.h_grid(V, np.arange(4).reshape(1, -1), 4)[0] + 1e-12


def test_gabriel_edges_half_length():
    # an edge whose open diametral ball holds no point of X has its midpoint
    # (a sample for even k) at distance |e|/2 from X, and that is the max
    X, L, cx = _small_problem(seed=5, n=40, nl=14)
    X64, L64 = X.astype(np.float64), L.astype(np.float64)
    E = cx["E"]
    f, _, _ = FL.flood_dim(X, L, E, 1, 4)
    hits = 0
    for i, (a, b) in enumerate(E):
        c = (L64[a] + L64[b]) / 2
        r = np.linalg.norm(L64[a] - L64[b]) / 2
        if np.all(np.linalg.norm(X64 - c, axis=1) >= r * (1 - 1e-9)):
            hits += 1
            assert abs(f[i] - r) <= 1e-12 * (1 + r)
    assert hits > 0


def test_stability_under_jitter():
    # Thm 2 (per simplex): |f_X - f_X'| <= d_H(X, X')
    X, L, cx = _small_problem(seed=0, n=500, nl=16)
    rng = np.random.default_rng(2)
    Xp = X.astype(np.float64) + rng.normal(0, 2e-3, X.shape)
    dH = np.linalg.norm(Xp - X, axis=1).max()  # bound on d_H via the matching
    for d, key in ((1, "E"), (2, "F"), (3, "T")):
        a, _, _ = FL.flood_dim(X, L, cx[key], d, 4)
        b, _, _ = FL.flood_dim(Xp, L, cx[key], d, 4)
        assert np.all(np.abs(a - b) <= dH * (1 + 1e-9))


def test_landmark_shift_bound():
    # samples move by at most max_i |dv_i| and d(., X) is 1-Lipschitz
    X, L, cx = _small_problem(seed=0, n=500, nl=16)
    rng = np.random.default_rng(3)
    Lp = L.astype(np.float64) + rng.normal(0, 1e-3, L.shape)
    for d, key in ((1, "E"), (2, "F"), (3, "T")):
        a, _, _ = FL.flood_dim(X, L, cx[key], d, 4)
        b, _, _ = FL.flood_dim(X, Lp, cx[key], d, 4)
        shift = np.linalg.norm(Lp - L, axis=1)[cx[key]].max(1)
        assert np.all(np.abs(a - b) <= shift * (1 + 1e-9))


def test_power_of_two_scaling_exact():
    X, L, cx = _small_problem()
    a = FL.flood_all(X, L, cx, 4)
    b = FL.flood_all(2.0 * X.astype(np.float64), 2.0 * L.astype(np.float64), cx, 4)
    for d in range(4):
        assert np.array_equal(2.0 * a[d][0], b[d][0])
        assert np.array_equal(a[d][2], b[d][2])


def test_circle_edge_sagitta():
    # Appendix circle example: an edge along an arc of angle a has value
    # 1 - cos(a/2) (its midpoint is the farthest sample, k even)
    N = 4096
    X = synth.circle_points(N)
    for nl in (8, 12):
        idx, _ = F.fps(X, nl)
        ang = np.sort(idx) * 2 * np.pi / N
        order = np.sort(idx)
        E = np.stack([order, np.roll(order, -1)], 1)
        E = np.sort(E, 1)
        arcs = (np.diff(np.concatenate([ang, [2 * np.pi]])))
        f, _, _ = FL.flood_dim(X, X, E, 1, 4)
        assert np.allclose(f, 1 - np.cos(arcs / 2), atol=1e-7)


# ---------------------------------------------------------------------------
# diam(X): every parity tolerance is 1e-5 * diam(X), so the oracle's diameter
# is pinned against brute force and shapes whose diameter is known.

def _diam_brute(X):
    X = np.asarray(X, np.float64)
    best = 0.0
    for i in range(len(X)):
        best = max(best, float(np.sqrt(((X[i] - X) ** 2).sum(1)).max()))
    return best


@pytest.mark.parametrize("seed", range(4))
def test_diameter_equals_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    clouds = [rng.random((300, 3)), rng.normal(size=(257, 3)) * [1.0, 0.3, 0.05],
              synth.config_cloud(1, n_points=400).astype(np.float64)]
    for X in clouds:
        assert abs(FL.diameter(X) - _diam_brute(X)) <= 1e-15 * _diam_brute(X)


def test_diameter_known_shapes():
    cube = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float64)
    assert abs(FL.diameter(cube) - np.sqrt(3.0)) <= 1e-15
    # collinear points (no hull): the two ends
    seg = np.outer(np.linspace(0.0, 2.5, 11), [0.6, 0.0, 0.8])
    assert abs(FL.diameter(seg) - 2.5) <= 1e-14
    # a sphere sample containing an antipodal pair: 2 r
    rng = np.random.default_rng(5)
    v = rng.normal(size=(200, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v[0], v[1] = [0, 0, 1], [0, 0, -1]
    assert abs(FL.diameter(0.7 * v) - 1.4) <= 1e-14
    # fewer than four points, and a single point
    assert abs(FL.diameter(cube[[0, 7]]) - np.sqrt(3.0)) <= 1e-15
    assert FL.diameter(cube[:1]) == 0.0
    # exact power-of-two scaling
    X = np.random.default_rng(6).random((100, 3))
    assert FL.diameter(4.0 * X) == 4.0 * FL.diameter(X)


def test_diameter_of_planar_clouds():
    # a planar cloud stored with z = 0 (ambient dimension 2): the hull is
    # taken in the plane; a cloud on a tilted plane falls back to all pairs
    P2 = synth.planar_cheese(500, 4, seed=7)
    X = np.zeros((len(P2), 3))
    X[:, :2] = P2
    assert abs(FL.diameter(X) - _diam_brute(X)) <= 1e-15 * _diam_brute(X)
    rng = np.random.default_rng(8)
    T = rng.random((300, 2)) @ np.array([[1.0, 0.2, 0.5], [0.1, 1.0, -0.3]])
    assert abs(FL.diameter(T) - _diam_brute(T)) <= 1e-15 * _diam_brute(T)


def test_diameter_of_the_torus_workload():
    # R = 1, r = 0.3: the outer equator has diameter 2 (R + r) = 2.6; the
    # noise (sigma = 0.01) moves it by a few sigma at most
    X = synth.config_cloud(1)
    assert 2.6 - 0.02 <= FL.diameter(X) <= 2.6 + 0.06


# ---------------------------------------------------------------------------
# Lemma 6 covering radius h(sigma), pinned from both sides: it must bound the
# grid's true covering radius (max over conv sigma of the distance to the
# nearest grid point), and on an edge and an equilateral triangle it exceeds
# it by exactly the factors 2 and 3 (closed forms of the 1-D grid and of the
# triangular lattice, whose covering radius is the small triangles'
# circumradius (l/k)/sqrt 3).

def _grid_cover_radius(V, k, n_probe):
    d = len(V) - 1
    A = FL.samples(d, k).astype(np.float64) / k
    G = A @ V
    rng = np.random.default_rng(9)
    lam = rng.dirichlet(np.ones(d + 1), n_probe)
    # dense probes plus the centroids of the grid's small cells
    fine = [FL.samples(d, m * k).astype(np.float64) / (m * k) for m in (3, 4)]
    P = np.concatenate([lam] + fine) @ V
    best = 0.0
    for i in range(0, len(P), 4096):
        dd = np.sqrt(((P[i:i + 4096, None, :] - G[None]) ** 2).sum(-1)).min(1)
        best = max(best, float(dd.max()))
    return best


def test_h_grid_closed_forms():
    for k in (1, 2, 3, 5, 8):
        e = np.array([[0.1, 0.2, 0.3], [1.3, -0.4, 0.5]])
        length = np.linalg.norm(e[1] - e[0])
        h = FL.h_grid(e, np.array([[0, 1]]), k)[0]
        assert abs(h - length / k) <= 1e-14
        assert abs(h - 2 * _grid_cover_radius(e, k, 2000)) <= 1e-12
        tri = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]]) * 0.75 + [0.2, 0.1, -0.3]
        h = FL.h_grid(tri, np.array([[0, 1, 2]]), k)[0]
        cov = _grid_cover_radius(tri, k, 20000)
        assert abs(h - 3 * cov) <= 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_h_grid_bounds_true_cover(seed):
    rng = np.random.default_rng(40 + seed)
    for d in (1, 2, 3):
        V = rng.random((d + 1, 3))
        for k in (2, 4):
            h = FL.h_grid(V, np.arange(d + 1).reshape(1, -1), k)[0]
            cov = _grid_cover_radius(V, k, 20000)
            assert cov <= h * (1 + 1e-12)
            # and between the longest edge over k and sqrt(#edges) times it
            emax = max(np.linalg.norm(V[i] - V[j]) for i in range(d + 1) for j in range(i))
            assert emax / k <= h * (1 + 1e-12) <= np.sqrt(d * (d + 1) / 2) * emax / k * (1 + 1e-12)
