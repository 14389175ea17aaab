"""Pins for the oracle's Delaunay triangulation and exact predicates."""
import numpy as np
import pytest

import synth
from oracle import delaunay as D
from oracle import fps as F
from oracle import predicates as P


def test_insphere_sign_convention():
    a, b, c, d = (np.array(v, float) for v in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 0]))
    o = P.orient_exact(a, b, c, d)
    assert o != 0
    assert P.insph_exact(a, b, c, d, [0.25, 0.25, 0.25]) * o > 0   # inside
    assert P.insph_exact(a, b, c, d, [2.0, 2.0, 2.0]) * o < 0      # outside
    assert P.insph_exact(a, b, c, d, [1.0, 1.0, 1.0]) == 0          # on (cube corner)
    s, fb = P.insph_sign(a, b, c, d, np.array([1.0, 1.0, 1.0]))
    assert s == 0 and fb == 1                                        # exact fallback used


def test_orient_exact_beyond_fp64():
    # nearly coplanar with a tiny offset that a naive float product rounds away
    a = np.array([0.1, 0.2, 0.3], np.float32)
    b = np.array([0.7, 0.1, 0.9], np.float32)
    c = np.array([0.3, 0.8, 0.2], np.float32)
    d = ((a.astype(np.float64) + b + c) / 3).astype(np.float32)
    s, _ = P.orient_sign(a, b, c, d)
    assert s == P.orient_exact(a, b, c, d)


@pytest.mark.parametrize("seed", range(4))
def test_brute_equals_qhull_equals_certified(seed):
    rng = np.random.default_rng(100 + seed)
    L = rng.random((24 + 4 * seed, 3)).astype(np.float32)
    B = D.brute_tets(L)
    assert np.array_equal(B, D.qhull_tets(L))
    D.certify(L, B)


def test_torus_landmarks_brute():
    X = synth.config_cloud(1)
    idx, _ = F.fps(X, 36)
    L = X[idx]
    B = D.brute_tets(L)
    assert np.array_equal(B, D.qhull_tets(L))
    D.certify(L, B)


def test_config1_certificate_and_euler():
    X = synth.config_cloud(1)
    idx, _ = F.fps(X, 64)
    L = X[idx]
    T = D.qhull_tets(L)
    info = D.certify(L, T)
    E, Fc, te, tt = D.faces(T)
    assert len(L) - len(E) + len(Fc) - len(T) == 1
    assert info["tets"] == len(T)
    # face maps: facet i omits vertex i
    for t in range(len(T)):
        for i in range(4):
            assert tuple(Fc[tt[t, i]]) == tuple(np.delete(T[t], i))
    for f in range(len(Fc)):
        for i in range(3):
            assert tuple(E[te[f, i]]) == tuple(np.delete(Fc[f], i))


def test_certificate_rejects_flipped_configuration():
    # five points: the 2-3 flip of a Delaunay pair is a valid triangulation
    # but not Delaunay; the certificate must reject it (planted mistake)
    P5 = np.array([[0, 0, 1], [1, 0, 0], [-0.5, 0.86, 0], [-0.5, -0.86, 0], [0, 0, -0.3]], np.float32)
    good = D.brute_tets(P5)
    D.certify(P5, good)
    two = [(0, 1, 2, 3), (4, 1, 2, 3)]
    three = [(0, 4, 1, 2), (0, 4, 2, 3), (0, 4, 3, 1)]
    bad = three if len(good) == 2 else two
    with pytest.raises(AssertionError):
        D.certify(P5, np.array(bad))


def test_certificate_rejects_missing_tet():
    rng = np.random.default_rng(7)
    L = rng.random((30, 3)).astype(np.float32)
    T = D.qhull_tets(L)
    with pytest.raises(AssertionError):
        D.certify(L, T[1:])


def test_degenerate_rejected():
    cube = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], np.float32)
    with pytest.raises(D.DegenerateInput):
        D.brute_tets(cube)


# ---------------------------------------------------------------- the plane

@pytest.mark.parametrize("seed", range(4))
def test_planar_brute_equals_qhull_and_certificate(seed):
    rng = np.random.default_rng(70 + seed)
    P = rng.random((12 + 6 * seed, 2)).astype(np.float32)
    F = D.brute_tris(P)
    assert np.array_equal(F, D.qhull_tris(P))
    info = D.certify2d(P, F)
    E, _ = D.faces2d(F)
    assert len(P) - len(E) + len(F) == 1 and info["triangles"] == len(F)


def test_planar_certificate_rejects_a_flipped_edge_and_a_missing_triangle():
    rng = np.random.default_rng(5)
    P = rng.random((25, 2)).astype(np.float32)
    F = [tuple(r) for r in D.brute_tris(P).tolist()]
    with pytest.raises(AssertionError):
        D.certify2d(P, np.array(F[1:]))
    for i in range(len(F)):
        for j in range(i + 1, len(F)):
            s = set(F[i]) & set(F[j])
            if len(s) != 2:
                continue
            a, b = sorted(s)
            c, d = (set(F[i]) - s).pop(), (set(F[j]) - s).pop()
            # the other diagonal of a convex quadrilateral
            G = [f for k, f in enumerate(F) if k not in (i, j)] + [tuple(sorted((a, c, d))), tuple(sorted((b, c, d)))]
            with pytest.raises(AssertionError):
                D.certify2d(P, np.array(G))
            return
    raise AssertionError("no shared edge found")


def test_planar_exact_predicates_decide_near_cocircular_points():
    # float32 points of a circle: every quadruple is nearly cocircular, so
    # the filter gives way to exact rational arithmetic
    OP = P
    t = 2 * np.pi * np.arange(8) / 8
    C = np.stack([np.cos(t), np.sin(t)], 1).astype(np.float32)
    s, fb = OP.incircle_sign(C[0], C[2], C[4], C[1:])
    assert fb > 0
    for k in range(1, 8):
        assert s[k - 1] == OP.incircle_exact(C[0], C[2], C[4], C[k])
    # the centre is inside, a far point outside (counter-clockwise triple)
    assert OP.incircle_exact([1, 0], [0, 1], [-1, 0], [0, 0]) == 1
    assert OP.incircle_exact([1, 0], [0, 1], [-1, 0], [0, -2]) == -1
    assert OP.orient2_exact([0, 0], [1, 0], [0, 1]) == 1
