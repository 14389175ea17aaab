"""Pins for the oracle's random sample sets (Thm. 5 with P_sigma drawn
uniformly from conv sigma, Lemma 9).

* the counter-based generator equals numpy's independent Philox4x64-10
  (numpy increments the counter before each block of four words);
* the barycentric weights are a point of the simplex, sum to 1 exactly, and
  are uniform on it (the marginal of a weight is Beta(1, d));
* every sample lies in conv sigma, so f_random <= r_exact (the exact value
  of Def. 1, from the Voronoi critical points); with many samples r_exact -
  f_random is small (Lemma 9);
* the closure is monotone, vertices of landmarks in X have f = 0, brute and
  Lemma-7-masked modes agree bit for bit;
* the analytic gradient equals FP64 central finite differences.
"""
import numpy as np
import pytest
from scipy import stats

import synth
from oracle import delaunay as D
from oracle import flood as FL
from oracle import fps as F


@pytest.mark.parametrize("key", [(0, 0), (5, 0), (0xdeadbeefcafef00d, 0x0123456789abcdef)])
@pytest.mark.parametrize("ctr", [(0, 0, 0, 0), (7, 11, 3, 0), (2 ** 64 - 1, 5, 2, 9)])
def test_philox_equals_numpy(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    want = bg.random_raw(4)
    # numpy generates the block of counter + 1 (with carry)
    c = list(ctr)
    c[0] = (c[0] + 1) % 2 ** 64
    if c[0] == 0:
        c[1] = (c[1] + 1) % 2 ** 64
    got = FL.philox4x64_10(c, key)
    assert np.array_equal(got, np.asarray(want, np.uint64))


def test_weights_on_the_simplex_and_exact():
    for d in (1, 2, 3):
        for q in range(200):
            w = FL.random_weights(d, q, 17, 99)
            assert len(w) == d + 1
            assert np.all(w >= 0) and w.sum() == 1.0
            # multiples of 2^-24: exact in float32 as well
            assert np.array_equal(w, w.astype(np.float32).astype(np.float64))
            assert np.all(np.round(w * 2 ** 24) == w * 2 ** 24)
    assert np.array_equal(FL.random_weights(0, 0, 3, 5), [1.0])


@pytest.mark.parametrize("d", [1, 2, 3])
def test_weights_uniform_on_the_simplex(d):
    # Dirichlet(1, ..., 1): every weight is Beta(1, d); draws over q and rows
    W = np.array([FL.random_weights(d, q, r, 2025) for r in range(40) for q in range(100)])
    for i in range(d + 1):
        p = stats.kstest(W[:, i], stats.beta(1, d).cdf).pvalue
        assert p > 1e-3, (d, i, p)
    assert np.abs(W.mean(0) - 1.0 / (d + 1)).max() < 0.02
    # different seeds, rows, samples and dimensions give different draws
    assert not np.array_equal(FL.random_weights(d, 0, 0, 1), FL.random_weights(d, 0, 0, 2))
    assert not np.array_equal(FL.random_weights(d, 0, 0, 1), FL.random_weights(d, 0, 1, 1))
    assert not np.array_equal(FL.random_weights(d, 0, 0, 1), FL.random_weights(d, 1, 0, 1))


@pytest.mark.parametrize("seed", range(4))
def test_random_samples_inside_the_hull(seed):
    # P_sigma inside conv sigma: f_random <= r_exact; and with many samples
    # the max over the hull is approached (Lemma 9)
    rng = np.random.default_rng(100 + seed)
    X = rng.random((14, 3))
    for d in (1, 2, 3):
        V = X[rng.choice(14, d + 1, replace=False)]
        r, _ = FL.r_exact(X, V)
        simp = np.arange(d + 1).reshape(1, -1)
        for m in (1, 7, 50):
            f, _, _ = FL.flood_random_dim(X, V, simp, d, m, seed)
            assert f[0] <= r + 1e-12, (d, m)
        f, _, _ = FL.flood_random_dim(X, V, simp, d, 20000, seed)
        diam_s = max(np.linalg.norm(V[i] - V[j]) for i in range(d + 1) for j in range(i + 1, d + 1))
        assert r - f[0] <= 0.05 * diam_s, (d, r, f[0])


def _complex(L):
    T = D.qhull_tets(L)
    E, Fc, te, tt = D.faces(T)
    return dict(E=E, F=Fc, T=T, tri_edges=te, tet_tris=tt, L=len(L))


def test_closure_vertices_and_masked():
    X = synth.config_cloud(1, n_points=600)
    idx, _ = F.fps(X, 20)
    L = X[idx]
    cx = _complex(L)
    m, seed = 16, 7
    vals = FL.flood_random_all(X, L, cx, m, seed)
    assert np.all(vals[0][0] == 0.0)
    f = FL.closure(vals, cx)
    assert np.all(f[0][cx["E"]].max(1) <= f[1])
    assert np.all(f[1][cx["tri_edges"]].max(1) <= f[2])
    assert np.all(f[2][cx["tet_tris"]].max(1) <= f[3])
    # unlike the nested grid, faces raise some values here
    assert any(np.any(f[d] > vals[d][0]) for d in (2, 3))
    masked = FL.flood_random_all(X, L, cx, m, seed, mode="masked")
    for d in range(4):
        for part in range(3):
            assert np.array_equal(vals[d][part], masked[d][part]), (d, part)
    # each own value is attained by its recorded sample and point
    simp = {1: cx["E"], 2: cx["F"], 3: cx["T"]}
    X64, L64 = X.astype(np.float64), L.astype(np.float64)
    for d in (1, 2, 3):
        for j in range(0, len(simp[d]), 7):
            w = FL.random_weights(d, int(vals[d][1][j]), j, seed)
            p = (w[:, None] * L64[simp[d][j]]).sum(0)
            dist = np.sqrt(((X64 - p) ** 2).sum(1))
            assert abs(dist.min() - vals[d][0][j]) <= 1e-12
            assert dist[vals[d][2][j]] == dist.min()


def test_random_gradient_matches_central_differences():
    X = synth.differentiable_clouds(1, 300, seed=79)[0].astype(np.float64)
    idx, _ = F.fps(X.astype(np.float32), 12)
    L = X[idx]
    cx = _complex(L)
    m, seed = 24, 3
    vals = FL.flood_random_all(X, L, cx, m, seed)
    rng = np.random.default_rng(1)
    w = {d: rng.random(len(vals[d][0])) for d in range(4)}
    gX, gL = FL.random_gradient(X, L, cx, vals, m, seed, w)

    def loss(XX, LL):
        v = FL.flood_random_all(XX, LL, cx, m, seed)
        f = FL.closure(v, cx)
        return sum((w[d] * f[d]).sum() for d in range(4))

    step = 1e-6
    for li in (0, 4, 9):
        for c in range(3):
            Lp, Lm = L.copy(), L.copy()
            Lp[li, c] += step
            Lm[li, c] -= step
            fd = (loss(X, Lp) - loss(X, Lm)) / (2 * step)
            assert abs(fd - gL[li, c]) <= 1e-4 * (1 + abs(fd)), (li, c, fd, gL[li, c])
    touched = np.flatnonzero(np.abs(gX).sum(1))[:6]
    assert len(touched) > 0
    for xi in touched:
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[xi, c] += step
            Xm[xi, c] -= step
            fd = (loss(Xp, L) - loss(Xm, L)) / (2 * step)
            assert abs(fd - gX[xi, c]) <= 1e-4 * (1 + abs(fd)), (xi, c, fd, gX[xi, c])
