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
