"""Pin for the oracle's analytic gradient: FP64 central finite differences."""
import numpy as np

import synth
from oracle import delaunay as D
from oracle import flood as FL
from oracle import fps as F


def _ties(X, L, simp, d, k, f):
    """Per simplex: gap between the two best samples and, at the best
    sample, between the two nearest points (FP64, small inputs)."""
    S = FL.samples(d, k) / k
    V = L[simp].astype(np.float64)
    P = np.einsum("sd,ndc->nsc", S, V)
    dist = np.sqrt(((P[:, :, None, :] - X[None, None].astype(np.float64)) ** 2).sum(-1))
    part = np.sort(dist, axis=-1)
    nn = part[..., 0]
    s_sorted = np.sort(nn, axis=1)
    sample_gap = s_sorted[:, -1] - s_sorted[:, -2] if nn.shape[1] > 1 else np.full(len(nn), np.inf)
    best = np.argmax(nn, axis=1)
    nn_gap = part[np.arange(len(nn)), best, 1] - part[np.arange(len(nn)), best, 0]
    return np.minimum(sample_gap, nn_gap)


def test_gradient_matches_central_differences():
    X = synth.differentiable_clouds(1, 400, seed=77)[0]
    idx, _ = F.fps(X, 14)
    L = X[idx]
    T = D.qhull_tets(L)
    E, Fc, te, tt = D.faces(T)
    cx = dict(E=E, F=Fc, T=T, tri_edges=te, tet_tris=tt)
    k = 4
    X64, L64 = X.astype(np.float64), L.astype(np.float64)
    diam = np.ptp(X64, 0).max()
    step = 1e-6
    checked = 0
    excluded = 0
    for d, simp in ((1, E), (2, Fc), (3, T)):
        f, wa, wx = FL.flood_dim(X64, L64, simp, d, k)
        gaps = _ties(X64, L64, simp, d, k, f)
        ok = gaps > 1e-5 * diam
        excluded += int((~ok).sum())
        sp = FL.winner_points(L64, simp, wa, k)
        u = (sp - X64[wx]) / f[:, None]
        # landmark coordinates
        for li in range(len(L)):
            for c in range(3):
                Lp, Lm = L64.copy(), L64.copy()
                Lp[li, c] += step
                Lm[li, c] -= step
                fd = (FL.flood_dim(X64, Lp, simp, d, k)[0] - FL.flood_dim(X64, Lm, simp, d, k)[0]) / (2 * step)
                an = ((simp == li) * (wa[:, : d + 1] / k)).sum(1) * u[:, c]
                assert np.allclose(fd[ok], an[ok], atol=1e-6, rtol=1e-5), (d, li, c)
                checked += int(ok.sum())
        # the argmin points' coordinates
        for xi in np.unique(wx)[:12]:
            for c in range(3):
                Xp, Xm = X64.copy(), X64.copy()
                Xp[xi, c] += step
                Xm[xi, c] -= step
                fd = (FL.flood_dim(Xp, L64, simp, d, k)[0] - FL.flood_dim(Xm, L64, simp, d, k)[0]) / (2 * step)
                an = -(wx == xi).astype(np.float64) * u[:, c]
                assert np.allclose(fd[ok], an[ok], atol=1e-6, rtol=1e-5), (d, xi, c)
    assert checked > 1000 and excluded < 0.2 * checked


def test_loss_gradient_assembles_per_simplex_terms():
    X = synth.differentiable_clouds(1, 300, seed=78)[0]
    idx, _ = F.fps(X, 12)
    L = X[idx]
    T = D.qhull_tets(L)
    E, Fc, te, tt = D.faces(T)
    cx = dict(E=E, F=Fc, T=T, tri_edges=te, tet_tris=tt)
    k = 4
    vals = FL.flood_all(X, L, cx, k)
    rng = np.random.default_rng(0)
    w = {d: rng.random(len(vals[d][0])) for d in range(4)}
    gX, gL = FL.gradient(X, L, cx, vals, k, w)
    # finite differences of the loss w.r.t. a few landmark coordinates
    loss = lambda LL: sum((w[d] * FL.flood_all(X, LL, cx, k)[d][0]).sum() for d in range(4))
    L64 = L.astype(np.float64)
    for li in (0, 3, 7):
        for c in range(3):
            Lp, Lm = L64.copy(), L64.copy()
            Lp[li, c] += 1e-6
            Lm[li, c] -= 1e-6
            fd = (loss(Lp) - loss(Lm)) / 2e-6
            assert abs(fd - gL[li, c]) <= 1e-4 * (1 + abs(fd))
