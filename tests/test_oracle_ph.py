"""Pins for the oracle's persistence computation and bottleneck test."""
import itertools
import os

import numpy as np
import pytest

import synth
from oracle import flood as FL
from oracle import fps as F
from oracle import ph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _closure_all(simplices):
    out = set()
    for s in simplices:
        for r in range(1, len(s) + 1):
            out.update(itertools.combinations(sorted(s), r))
    return out


def test_textbook_complexes():
    # hollow tetrahedron: one H2 class; triangle boundary: one H1 class
    hollow = sorted(_closure_all(itertools.combinations(range(4), 3)), key=lambda s: (len(s), s))
    pairs, ess = ph.reduce_pairs(hollow, [len(s) - 1 for s in hollow])
    assert sorted(len(hollow[i]) - 1 for i in ess) == [0, 2]
    ring = sorted(_closure_all([(0, 1), (1, 2), (0, 2)]), key=lambda s: (len(s), s))
    pairs, ess = ph.reduce_pairs(ring, [len(s) - 1 for s in ring])
    assert sorted(len(ring[i]) - 1 for i in ess) == [0, 1]


@pytest.mark.parametrize("seed", range(6))
def test_reduction_equals_rank_invariant(seed):
    rng = np.random.default_rng(seed)
    pts = rng.random((7, 3))
    from scipy.spatial import Delaunay
    T = Delaunay(pts).simplices
    cl = list(_closure_all([tuple(t) for t in T]))
    vals = {s: rng.random() for s in cl}
    # make the values monotone (a filtration)
    for s in sorted(cl, key=len):
        for r in range(1, len(s)):
            for f in itertools.combinations(s, r):
                vals[s] = max(vals[s], vals[f])
    order = sorted(cl, key=lambda s: (vals[s], len(s), s))
    dims = [len(s) - 1 for s in order]
    pairs, ess = ph.reduce_pairs(order, dims)
    got = {p: [] for p in range(3)}
    for i, j in pairs:
        got[dims[i]].append((i, j))
    for i in ess:
        if dims[i] <= 2:
            got[dims[i]].append((i, None))
    ref = ph.rank_invariant_pairs(order, dims)
    for p in range(3):
        key = lambda t: (t[0], -1 if t[1] is None else t[1])
        assert sorted(got[p], key=key) == ref[p]


def test_bottleneck_threshold():
    A = (np.array([[0.0, 1.0], [0.2, 0.3]]), np.array([0.0]))
    B = (np.array([[0.0, 1.05]]), np.array([0.01]))
    assert ph.bottleneck_leq(A, A, 0.0)
    # (0.2,0.3) must go to the diagonal: cost 0.05; (0,1)->(0,1.05): 0.05
    assert ph.bottleneck_leq(A, B, 0.05 + 1e-12)
    assert not ph.bottleneck_leq(A, B, 0.049)
    C = (np.zeros((0, 2)), np.array([0.0, 0.5]))
    assert not ph.bottleneck_leq(A, C, 10.0)  # essential counts differ


def _polygon_complex(order):
    n = len(order)
    E = {tuple(sorted((order[i], order[(i + 1) % n]))) for i in range(n)}
    Fs = set()
    for i in range(1, n - 1):
        t = tuple(sorted((order[0], order[i], order[i + 1])))
        Fs.add(t)
        E.update({tuple(sorted(p)) for p in itertools.combinations(t, 2)})
    E = np.array(sorted(E))
    Fs = np.array(sorted(Fs))
    ekey = {tuple(e): i for i, e in enumerate(E.tolist())}
    te = np.array([[ekey[(f[1], f[2])], ekey[(f[0], f[2])], ekey[(f[0], f[1])]] for f in Fs.tolist()])
    return E, Fs, te


def test_circle_diagrams_golden():
    # Appendix circle example, on a fan triangulation of the landmark polygon
    # (the diagrams do not depend on which triangulation is used).
    N = 4096
    X = synth.circle_points(N)
    for line in open(os.path.join(GOLDEN, "circle_example.txt")):
        if line.startswith("#") or not line.strip():
            continue
        nl, m, phi_pi = line.split()
        nl, m, phi = int(nl), int(m), float(phi_pi) * np.pi
        idx, _ = F.fps(X, nl)
        order = np.sort(idx)
        E, Fs, te = _polygon_complex(list(range(nl)))
        Lxyz = X[order]
        k = 8
        fv = FL.flood_dim(X, Lxyz, np.arange(nl).reshape(-1, 1), 0, k)[0]
        fe = FL.flood_dim(X, Lxyz, E, 1, k)[0]
        ff = FL.flood_dim(X, Lxyz, Fs, 2, k)[0]
        fe = np.maximum(fe, 0)
        ff = np.maximum(ff, fe[te].max(1))
        cx = dict(L=nl, E=E, F=Fs, T=np.zeros((0, 4), int))
        dg = ph.diagrams(cx, {0: fv, 1: fe, 2: ff, 3: np.zeros(0)}, maxdim=1)
        tol = 2e-3  # triangle samples are within h of the centre
        short, long_ = 1 - np.cos(phi / 2), 1 - np.cos(phi)
        # H0: m short arcs, the long arcs but the one that closes the cycle
        want0 = np.array([[0, short]] * m + [[0, long_]] * (nl - m - 1)).reshape(-1, 2)
        assert ph.bottleneck_leq(dg[0], (want0, np.array([0.0])), 1e-6)  # float32 circle points
        want1 = np.array([[long_ if m < nl else short, 1.0]])
        assert ph.bottleneck_leq(dg[1], (want1, np.zeros(0)), tol)
