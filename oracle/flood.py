"""Sampled flood values and their derivatives (oracle; test infrastructure).

Definitions followed (paper sections named, not copied):
* Def. 1: sigma is in Flood_r(X, L) iff conv(sigma) is inside the union of
  r-balls around X, so f(sigma) = max_{p in conv sigma} min_{x in X} ||p-x||
  (Sec. 4.1: the directed Hausdorff distance from conv sigma to X).
* Sec. 4.1, sampled complex: f_P(sigma) = max over faces tau of sigma of
  max_{p in P_tau} d(p, X).
* Lemma 6: P_sigma = { sum_i (a_i/k) v_i : a_i in N, sum a_i = k } (k
  segments, k+1 points per edge); d_H(P_sigma, conv sigma) <=
  sqrt(sum_{i<j} ||v_i - v_j||^2) / k.
* Lemma 7: with L inside X, the nearest point of X to any p in conv sigma
  lies in B(c, sqrt(2) r) for an enclosing ball B(c, r) of sigma; the ball
  used is the midpoint of the longest edge (radius without sqrt(2) for an
  edge), as Sec. 4.2 describes.

The value computations run in the C part (flood_oracle.c) in FP64.
"""
from itertools import combinations

import numpy as np

from . import native


def _as_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class XSorted:
    """X presorted along the first axis, for masked mode (Sec. 4.2 appendix:
    presort + binary search per simplex)."""

    def __init__(self, X):
        X = _as_f64(X)
        self.order = np.ascontiguousarray(np.argsort(X[:, 0], kind="stable").astype(np.int64))
        self.xs = np.ascontiguousarray(X[self.order])


def samples(d: int, k: int) -> np.ndarray:
    """The compositions a (rows, d+1 entries summing to k) in the order the
    C part visits them (lexicographically descending)."""
    n = native.lib().or_count_samples(d, k, None)
    out = np.zeros((n, d + 1), np.int32)
    native.lib().or_count_samples(d, k, native.ptr(out))
    return out


def landmarks_in_x(X, Lxyz) -> bool:
    """True if every landmark coordinate is (bit-exactly) a point of X."""
    Xv = np.ascontiguousarray(X, dtype=np.float64).view([("", np.float64)] * 3).ravel()
    Lv = np.ascontiguousarray(Lxyz, dtype=np.float64).view([("", np.float64)] * 3).ravel()
    return bool(np.all(np.isin(Lv, Xv)))


def flood_dim(X, Lxyz, simp, d: int, k: int, mode: str = "brute", xsorted=None, nthreads=None, counter=None,
              gaps=False):
    """f_P(sigma) for the d-simplices `simp` ([n, d+1] landmark ids), without
    the face closure.  Returns (f float64 [n], win_a int32 [n,4], win_x int32 [n]).
    `counter` (int64 numpy array of one element) accumulates the number of
    distance evaluations performed.  With gaps=True also returns
    (gap between the two best samples, gap between the two nearest points at
    the best sample) per simplex."""
    X = _as_f64(X)
    Lxyz = _as_f64(Lxyz)
    simp = np.ascontiguousarray(simp, dtype=np.int32).reshape(-1, d + 1)
    n = simp.shape[0]
    f = np.zeros(n, np.float64)
    wa = np.zeros((n, 4), np.int32)
    wx = np.zeros(n, np.int32)
    gs = np.zeros(n, np.float64)
    gx = np.zeros(n, np.float64)
    if n == 0:
        return (f, wa, wx, gs, gx) if gaps else (f, wa, wx)
    m = {"brute": 0, "masked": 1}[mode]
    if m == 1 and xsorted is None:
        xsorted = XSorted(X)
    xs = xsorted.xs if m == 1 else X
    order = xsorted.order if m == 1 else np.zeros(1, np.int64)
    rc = native.lib().or_flood(native.ptr(X), X.shape[0], native.ptr(Lxyz), native.ptr(simp), n,
                               d, k, m, native.ptr(xs), native.ptr(order), native.ptr(f),
                               native.ptr(wa), native.ptr(wx),
                               native.ptr(counter) if counter is not None else None,
                               native.ptr(gs) if gaps else None, native.ptr(gx) if gaps else None,
                               native.threads(nthreads))
    if rc != 0:
        raise ValueError("or_flood failed: %d" % rc)
    return (f, wa, wx, gs, gx) if gaps else (f, wa, wx)


def flood_all(X, Lxyz, cx, k: int, mode: str = "brute", nthreads=None):
    """Flood values for a whole complex.  cx: dict with 'E','F','T' (sorted
    rows of landmark ids).  Returns {d: (f, win_a, win_x)} for d = 0..3;
    vertices are the 0-simplices 0..L-1."""
    Lxyz = _as_f64(Lxyz)
    xsorted = XSorted(X) if mode == "masked" else None
    simp = {0: np.arange(Lxyz.shape[0]).reshape(-1, 1), 1: cx["E"], 2: cx["F"], 3: cx["T"]}
    return {d: flood_dim(X, Lxyz, simp[d], d, k, mode, xsorted, nthreads) for d in range(4)}


def closure(vals, cx):
    """Monotone closure f(sigma) = max(f_P(sigma), max over facets f(tau))
    (Sec. 4.1, the sampled complex requires every face to be flooded).
    Returns {d: f} with the closure applied bottom-up."""
    out = {0: vals[0][0].copy()}
    E, F = cx["E"], cx["F"]
    fE = np.maximum(vals[1][0], np.maximum(out[0][E[:, 0]], out[0][E[:, 1]])) if len(E) else vals[1][0].copy()
    out[1] = fE
    out[2] = np.maximum(vals[2][0], out[1][cx["tri_edges"]].max(1)) if len(F) else vals[2][0].copy()
    out[3] = np.maximum(vals[3][0], out[2][cx["tet_tris"]].max(1)) if len(cx["T"]) else vals[3][0].copy()
    return out


def assert_closure_noop(vals, cx):
    """With the full nested grid (P_tau a subset of P_sigma, bit-identical
    coordinates) the closure changes nothing; assert it."""
    c = closure(vals, cx)
    for d in range(4):
        assert np.array_equal(c[d], vals[d][0]), "closure changed dimension %d" % d
    return c


def h_grid(Lxyz, simp, k: int):
    """Lemma 6 covering radius of the barycentric grid: sqrt(sum_{i<j} ||v_i-v_j||^2)/k."""
    V = _as_f64(Lxyz)[np.asarray(simp)]
    s = np.zeros(V.shape[0])
    for i, j in combinations(range(V.shape[1]), 2):
        s += ((V[:, i] - V[:, j]) ** 2).sum(1)
    return np.sqrt(s) / k


def winner_points(Lxyz, simp, win_a, k):
    """The argmax sample s* = sum_i (a_i/k) v_i (FP64, same order as the C part)."""
    V = _as_f64(Lxyz)[np.asarray(simp)]
    p = np.zeros((V.shape[0], 3))
    for i in range(V.shape[1]):
        p = p + (win_a[:, i:i + 1] / k) * V[:, i]
    return p


def gradient(X, Lxyz, cx, vals, k, weights):
    """Analytic gradient of loss = sum_d sum_sigma w_sigma f(sigma).

    f(sigma) = ||s* - x*|| with s* = sum_i (a*_i/k) v_i the argmax sample and
    x* its nearest point; away from ties, df = u . (ds* - dx*) with
    u = (s* - x*)/f.  Hence dL/dx* -= w u and dL/dv_i += w (a*_i/k) u; u = 0
    when f = 0.  weights: {d: w [n_d]}.  Returns (gX [N,3], gL [L,3])."""
    X = _as_f64(X)
    Lxyz = _as_f64(Lxyz)
    gX = np.zeros_like(X)
    gL = np.zeros_like(Lxyz)
    simp = {0: np.arange(Lxyz.shape[0]).reshape(-1, 1), 1: cx["E"], 2: cx["F"], 3: cx["T"]}
    for d in range(4):
        f, wa, wx = vals[d]
        w = np.asarray(weights[d], dtype=np.float64)
        if len(f) == 0:
            continue
        sp = winner_points(Lxyz, simp[d], wa, k)
        diff = sp - X[wx]
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(f[:, None] > 0, diff / f[:, None], 0.0)
        np.add.at(gX, wx, -w[:, None] * u)
        for i in range(d + 1):
            np.add.at(gL, simp[d][:, i], w[:, None] * (wa[:, i:i + 1] / k) * u)
    return gX, gL


def r_exact(X, V):
    """Exact f(sigma) = max_{p in conv sigma} d(p, X) for one simplex with
    vertex coordinates V [d+1, 3] (tiny X only).

    d(., X) restricted to conv(sigma) is, on each piece (Voronoi cell of x)
    cap (face of sigma), the convex function ||p - x||; its maximum sits at
    a vertex of that piece.  Such a vertex lies in the relative interior of
    some face phi of sigma (dim j) and is equidistant from j+1 points S of X
    that are its nearest points.  Enumerate (phi, S), solve the j x j linear
    system for p in aff(phi), keep p if it is inside phi and S attains
    d(p, X); return the max (and the candidate count)."""
    X = _as_f64(X)
    V = _as_f64(V)
    n = len(X)
    diam = max(np.ptp(X, 0).max(), 1e-300)
    best, cnt = 0.0, 0
    for j in range(V.shape[0]):
        for phi in combinations(range(V.shape[0]), j + 1):
            F = V[list(phi)]
            B = (F[1:] - F[0]).T  # 3 x j
            for S in combinations(range(n), j + 1):
                Sx = X[list(S)]
                if j == 0:
                    p = F[0]
                else:
                    # 2 p.(s_i - s_0) = |s_i|^2 - |s_0|^2, p = F0 + B mu
                    A = 2.0 * (Sx[1:] - Sx[0])  # j x 3
                    rhs = (Sx[1:] ** 2).sum(1) - (Sx[0] ** 2).sum() - A @ F[0]
                    M = A @ B
                    if abs(np.linalg.det(M)) < 1e-14 * max(1.0, np.abs(M).max() ** j):
                        continue
                    mu = np.linalg.solve(M, rhs)
                    lam = np.concatenate([[1.0 - mu.sum()], mu])
                    if lam.min() < -1e-12:
                        continue
                    p = F[0] + B @ mu
                dall = np.sqrt(((X - p) ** 2).sum(1))
                dmin = dall.min()
                if dall[list(S)].max() <= dmin + 1e-12 * diam:
                    cnt += 1
                    best = max(best, dmin)
    return best, cnt


def diameter(X) -> float:
    """diam(X): the largest pairwise distance, exactly over the convex-hull
    vertices (FP64).  Coordinates that are constant over X (a planar cloud
    stored with z = 0) are left out of the hull, which then lives in the
    remaining coordinates; the distances are unchanged."""
    X = _as_f64(X)
    Xh = X[:, np.ptp(X, axis=0) > 0] if len(X) else X
    if len(X) <= 3 or Xh.shape[1] == 0:
        idx = np.arange(len(X))
    elif Xh.shape[1] == 1:
        idx = np.array([int(np.argmin(Xh[:, 0])), int(np.argmax(Xh[:, 0]))])
    else:
        from scipy.spatial import ConvexHull
        try:
            idx = ConvexHull(Xh).vertices
        except Exception:
            idx = np.arange(len(X))
    H = X[idx]
    best = 0.0
    for i in range(0, len(H), 512):
        d = ((H[i:i + 512, None, :] - H[None, :, :]) ** 2).sum(-1)
        best = max(best, float(d.max()))
    return float(np.sqrt(best))


def nearest(X, P):
    """Distance from each row of P to X and the lowest-index nearest point
    (brute force, FP64; small inputs)."""
    X = _as_f64(X)
    P = _as_f64(P)
    out_d = np.empty(len(P))
    out_i = np.empty(len(P), np.int64)
    for i in range(0, len(P), 256):
        d = ((P[i:i + 256, None, :] - X[None]) ** 2).sum(-1)
        out_i[i:i + 256] = np.argmin(d, axis=1)
        out_d[i:i + 256] = np.sqrt(d[np.arange(len(d)), out_i[i:i + 256]])
    return out_d, out_i


# ---------------------------------------------------------------------------
# Random sample sets (Thm. 5 for any P_sigma inside conv sigma; Lemma 9 for
# uniform draws).  Each simplex of dimension >= 1 owns m points drawn from
# its convex hull by a counter-based generator (see flood_oracle.c); each
# face has its own set, so the closure over faces is load-bearing.


def philox4x64_10(ctr, key):
    """The raw generator of the C part: 4 words for counter `ctr` (4 uint64)
    and key `key` (2 uint64)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    native.lib().or_philox4x64_10(native.ptr(c), native.ptr(k), native.ptr(out))
    return out


def random_weights(d: int, q: int, row: int, seed: int) -> np.ndarray:
    """Barycentric weights (d+1 entries) of random sample q of the simplex in
    cloud-local row `row` of dimension d."""
    w = np.zeros(4, np.float64)
    native.lib().or_random_weights(d, q, row, seed, native.ptr(w))
    return w[:d + 1].copy()


def flood_random_dim(X, Lxyz, simp, d: int, m: int, seed: int, rows=None, mode: str = "brute", xsorted=None,
                     nthreads=None, counter=None):
    """Own value of each d-simplex under random sample sets (max over its m
    samples of d(p, X); vertices: the vertex), without the face closure.
    rows: the simplices' cloud-local rows (default 0..n-1).  Returns
    (f float64 [n], win_q int32 [n], win_x int32 [n])."""
    X = _as_f64(X)
    Lxyz = _as_f64(Lxyz)
    simp = np.ascontiguousarray(simp, dtype=np.int32).reshape(-1, d + 1)
    n = simp.shape[0]
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    f = np.zeros(n, np.float64)
    wq = np.zeros(n, np.int32)
    wx = np.zeros(n, np.int32)
    if n == 0:
        return f, wq, wx
    md = {"brute": 0, "masked": 1}[mode]
    if md == 1 and xsorted is None:
        xsorted = XSorted(X)
    xs = xsorted.xs if md == 1 else X
    order = xsorted.order if md == 1 else np.zeros(1, np.int64)
    rc = native.lib().or_flood_random(native.ptr(X), X.shape[0], native.ptr(Lxyz), native.ptr(simp),
                                      native.ptr(rows), n, d, m, seed, md, native.ptr(xs), native.ptr(order),
                                      native.ptr(f), native.ptr(wq), native.ptr(wx),
                                      native.ptr(counter) if counter is not None else None,
                                      native.threads(nthreads))
    if rc != 0:
        raise ValueError("or_flood_random failed: %d" % rc)
    return f, wq, wx


def flood_random_all(X, Lxyz, cx, m: int, seed: int, mode: str = "brute", nthreads=None):
    """Own values of every simplex under random sample sets: {d: (f, win_q,
    win_x)}; apply `closure` for the filtration."""
    Lxyz = _as_f64(Lxyz)
    xsorted = XSorted(X) if mode == "masked" else None
    simp = {0: np.arange(Lxyz.shape[0]).reshape(-1, 1), 1: cx["E"], 2: cx["F"], 3: cx["T"]}
    return {d: flood_random_dim(X, Lxyz, simp[d], d, m, seed, None, mode, xsorted, nthreads) for d in range(4)}


def random_winners(vals, cx):
    """For the closure f(sigma) = max(own(sigma), max over facets f(tau)):
    the simplex (dimension, row) that owns the winning sample of every
    simplex -- its own sample when own >= the facets' max, else the first
    facet (omitting vertex i, i ascending) attaining the max, followed down.
    Returns {d: (owner_dim [n], owner_row [n])}."""
    f = closure(vals, cx)
    facets = {1: None, 2: cx["tri_edges"], 3: cx["tet_tris"]}
    own = {}
    own[0] = (np.zeros(len(f[0]), np.int64), np.arange(len(f[0]), dtype=np.int64))
    for d in (1, 2, 3):
        n = len(f[d])
        od = np.full(n, d, np.int64)
        orow = np.arange(n, dtype=np.int64)
        for j in range(n):
            if vals[d][0][j] >= f[d][j]:
                continue
            if d == 1:
                fac = [cx["E"][j][1], cx["E"][j][0]]  # facet i omits vertex i
            else:
                fac = list(facets[d][j])
            for i, t in enumerate(fac):
                if f[d - 1][t] == f[d][j]:
                    od[j], orow[j] = own[d - 1][0][t], own[d - 1][1][t]
                    break
        own[d] = (od, orow)
    return own


def random_gradient(X, Lxyz, cx, vals, m, seed, weights):
    """Analytic gradient of loss = sum_sigma w_sigma f(sigma) under random
    sample sets: the winning sample s* = sum_i w*_i v_i belongs to the owner
    simplex (random_winners), x* is its nearest point; dL/dx* -= w u,
    dL/dv_i += w w*_i u over the owner's vertices, u = (s* - x*)/f."""
    X = _as_f64(X)
    Lxyz = _as_f64(Lxyz)
    gX = np.zeros_like(X)
    gL = np.zeros_like(Lxyz)
    simp = {0: np.arange(Lxyz.shape[0]).reshape(-1, 1), 1: cx["E"], 2: cx["F"], 3: cx["T"]}
    f = closure(vals, cx)
    own = random_winners(vals, cx)
    for d in range(4):
        w = np.asarray(weights[d], dtype=np.float64)
        for j in range(len(f[d])):
            if w[j] == 0.0 or f[d][j] <= 0.0:
                continue
            od, orow = int(own[d][0][j]), int(own[d][1][j])
            q = int(vals[od][1][orow])
            xi = int(vals[od][2][orow])
            bw = random_weights(od, q, orow, seed)
            vv = simp[od][orow]
            sp = (bw[:, None] * Lxyz[vv]).sum(0)
            u = (sp - X[xi]) / f[d][j]
            gX[xi] -= w[j] * u
            for i in range(od + 1):
                gL[vv[i]] += w[j] * bw[i] * u
    return gX, gL
