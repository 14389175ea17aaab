"""Delaunay triangulation of the landmarks (oracle; test infrastructure).

Del(L) is the complex on which the filtration lives (Sec. 3 and Sec. 4,
"Computational aspects").  The paper assumes general position; inputs with
an exactly coplanar tetrahedron candidate or exactly cospherical 5-tuple in
play are rejected here (DegenerateInput).

* ``brute_tets``: every 4-subset with non-zero orientation whose open
  circumsphere contains no other landmark (the empty-sphere definition).
  O(L^5); tiny inputs only.
* ``certify``: checks that a given tetrahedron list is the Delaunay
  triangulation of L: each tet non-degenerate; each triangle in one or two
  tets; the two tets of an interior triangle lie on opposite sides of it and
  neither's opposite vertex is inside the other's circumsphere (locally
  Delaunay); every hull triangle has all landmarks on its tet's side; every
  landmark is used.  A locally Delaunay triangulation of the hull is the
  Delaunay triangulation (Delaunay's lemma), unique in general position.
* ``faces``: the closure -- sorted edge and triangle lists and face maps.
* In the plane (ambient dimension 2, Sec. 5.2): ``brute_tris`` (empty
  circumcircles), ``certify2d`` (every interior edge locally Delaunay, hull
  edges supporting, Euler characteristic 1) and ``faces2d``.
"""
from itertools import combinations

import numpy as np

from .predicates import incircle_sign, insph_sign, orient2_sign, orient_sign


class DegenerateInput(ValueError):
    pass


def brute_tets(P: np.ndarray) -> np.ndarray:
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    quads = np.array(list(combinations(range(n), 4)), dtype=np.int64)
    o, _ = orient_sign(P[quads[:, 0]], P[quads[:, 1]], P[quads[:, 2]], P[quads[:, 3]])
    if np.any(o == 0):
        raise DegenerateInput("coplanar 4-subset")
    keep = []
    for lo in range(0, len(quads), 4096):
        q = quads[lo:lo + 4096]
        oo = o[lo:lo + 4096].astype(np.int64)
        a, b, c, d = (P[q[:, i]][:, None, :] for i in range(4))
        e = P[None, :, :]
        member = np.zeros((len(q), n), dtype=bool)
        member[np.arange(len(q))[:, None], q] = True
        s, _ = insph_sign(a, b, c, d, e, skip=member)
        inside = s.astype(np.int64) * oo[:, None]
        on = (s == 0) & ~member
        if np.any(on):
            raise DegenerateInput("cospherical 5-subset")
        empty = ~np.any((inside > 0) & ~member, axis=1)
        keep.append(q[empty])
    T = np.concatenate(keep) if keep else np.zeros((0, 4), np.int64)
    return canonical(T)


def canonical(T: np.ndarray) -> np.ndarray:
    T = np.sort(np.asarray(T, dtype=np.int64), axis=1)
    if len(T) == 0:
        return T.reshape(0, 4)
    order = np.lexsort(T.T[::-1])
    return T[order]


def faces(T: np.ndarray):
    """Returns (E [nE,2], F [nF,3], tri_edges [nF,3], tet_tris [nT,4]), all
    rows sorted, lexicographically ordered; facet i of a simplex is the one
    without its i-th vertex."""
    T = canonical(T)
    tri_sets = [T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]]
    F = np.unique(np.concatenate(tri_sets), axis=0)
    edge_sets = [F[:, [1, 2]], F[:, [0, 2]], F[:, [0, 1]]]
    E = np.unique(np.concatenate(edge_sets), axis=0)
    fkey = {tuple(r): i for i, r in enumerate(F.tolist())}
    ekey = {tuple(r): i for i, r in enumerate(E.tolist())}
    tet_tris = np.array([[fkey[tuple(s[i])] for s in tri_sets] for i in range(len(T))],
                        dtype=np.int64).reshape(-1, 4)
    tri_edges = np.array([[ekey[tuple(s[i])] for s in edge_sets] for i in range(len(F))],
                         dtype=np.int64).reshape(-1, 3)
    return E, F, tri_edges, tet_tris


def certify(P: np.ndarray, T: np.ndarray) -> dict:
    """Raises AssertionError unless T is the Delaunay triangulation of P."""
    P = np.asarray(P, dtype=np.float64)
    T = canonical(T)
    n = P.shape[0]
    o, fb0 = orient_sign(P[T[:, 0]], P[T[:, 1]], P[T[:, 2]], P[T[:, 3]])
    assert np.all(o != 0), "degenerate tetrahedron"
    # triangle -> incident (tet, opposite vertex)
    tri = np.concatenate([T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]])
    opp = np.concatenate([T[:, 0], T[:, 1], T[:, 2], T[:, 3]])
    tet = np.concatenate([np.arange(len(T))] * 4)
    key = np.lexsort(tri.T[::-1])
    tri, opp, tet = tri[key], opp[key], tet[key]
    same_next = np.all(tri[1:] == tri[:-1], axis=1)
    # no triangle in three tets
    assert not np.any(same_next[1:] & same_next[:-1]), "triangle in more than two tets"
    first = np.flatnonzero(np.concatenate([[True], ~same_next]))
    count = np.diff(np.concatenate([first, [len(tri)]]))
    inner = first[count == 2]
    hull = first[count == 1]
    # interior triangles: opposite vertices on opposite sides, locally Delaunay
    t = tri[inner]
    a, b, c = P[t[:, 0]], P[t[:, 1]], P[t[:, 2]]
    s1, fb1 = orient_sign(a, b, c, P[opp[inner]])
    s2, fb2 = orient_sign(a, b, c, P[opp[inner + 1]])
    assert np.all(s1 * s2 < 0), "tets on the same side of a shared triangle"
    # opposite vertex of tet 2 not inside circumsphere of tet 1
    T1 = T[tet[inner]]
    oo, _ = orient_sign(P[T1[:, 0]], P[T1[:, 1]], P[T1[:, 2]], P[T1[:, 3]])
    si, fb3 = insph_sign(P[T1[:, 0]], P[T1[:, 1]], P[T1[:, 2]], P[T1[:, 3]], P[opp[inner + 1]])
    ins = si.astype(np.int64) * oo
    assert np.all(ins < 0), "not locally Delaunay (or cospherical)"
    # hull triangles: every landmark on the side of the tet (or on the plane
    # only if it is a vertex of the triangle)
    h = tri[hull]
    side, _ = orient_sign(P[h[:, 0]], P[h[:, 1]], P[h[:, 2]], P[opp[hull]])
    fbh = 0
    for lo in range(0, len(h), 256):
        hh = h[lo:lo + 256]
        ss = side[lo:lo + 256].astype(np.int64)
        member = np.zeros((len(hh), n), dtype=bool)
        member[np.arange(len(hh))[:, None], hh] = True
        sgn, fb = orient_sign(P[hh[:, 0]][:, None], P[hh[:, 1]][:, None], P[hh[:, 2]][:, None],
                              P[None, :, :], skip=member)
        fbh += fb
        bad = (sgn.astype(np.int64) * ss[:, None] < 0) | ((sgn == 0) & ~member)
        assert not np.any(bad), "hull triangle is not a supporting plane"
    assert len(np.unique(T)) == n, "landmark missing from the triangulation"
    E, F, _, _ = faces(T)
    euler = n - len(E) + len(F) - len(T)
    assert euler == 1, "Euler characteristic %d" % euler
    return {"tets": len(T), "hull_triangles": len(hull), "exact_fallbacks": fb0 + fb1 + fb2 + fb3 + fbh}


def qhull_tets(P: np.ndarray) -> np.ndarray:
    """scipy's qhull Delaunay, canonicalised -- an independent cross-check."""
    from scipy.spatial import Delaunay
    return canonical(Delaunay(np.asarray(P, dtype=np.float64)).simplices)


# --------------------------------------------------------------------------
# the plane


def canonical2(F: np.ndarray) -> np.ndarray:
    F = np.sort(np.asarray(F, dtype=np.int64), axis=1)
    if len(F) == 0:
        return F.reshape(0, 3)
    return F[np.lexsort(F.T[::-1])]


def brute_tris(P: np.ndarray) -> np.ndarray:
    """Every triple with non-zero orientation whose open circumcircle holds
    no other point.  O(L^4); tiny inputs only."""
    P = np.asarray(P, dtype=np.float64)
    n = P.shape[0]
    tri = np.array(list(combinations(range(n), 3)), dtype=np.int64)
    o, _ = orient2_sign(P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]])
    if np.any(o == 0):
        raise DegenerateInput("collinear triple")
    member = np.zeros((len(tri), n), dtype=bool)
    member[np.arange(len(tri))[:, None], tri] = True
    s, _ = incircle_sign(P[tri[:, 0]][:, None], P[tri[:, 1]][:, None], P[tri[:, 2]][:, None], P[None, :, :],
                         skip=member)
    inside = s.astype(np.int64) * o.astype(np.int64)[:, None]
    if np.any((s == 0) & ~member):
        raise DegenerateInput("cocircular 4-subset")
    empty = ~np.any((inside > 0) & ~member, axis=1)
    return canonical2(tri[empty])


def faces2d(F: np.ndarray):
    """(E [nE,2], tri_edges [nF,3]) of a triangle list, rows sorted; edge i of
    a triangle is the one without its i-th vertex."""
    F = canonical2(F)
    edge_sets = [F[:, [1, 2]], F[:, [0, 2]], F[:, [0, 1]]]
    E = np.unique(np.concatenate(edge_sets), axis=0)
    ekey = {tuple(r): i for i, r in enumerate(E.tolist())}
    tri_edges = np.array([[ekey[tuple(s[i])] for s in edge_sets] for i in range(len(F))],
                         dtype=np.int64).reshape(-1, 3)
    return E, tri_edges


def certify2d(P: np.ndarray, F: np.ndarray) -> dict:
    """Raises AssertionError unless F is the Delaunay triangulation of the
    planar points P (Delaunay's lemma in the plane)."""
    P = np.asarray(P, dtype=np.float64)
    F = canonical2(F)
    n = P.shape[0]
    o, fb0 = orient2_sign(P[F[:, 0]], P[F[:, 1]], P[F[:, 2]])
    assert np.all(o != 0), "degenerate triangle"
    edge = np.concatenate([F[:, [1, 2]], F[:, [0, 2]], F[:, [0, 1]]])
    opp = np.concatenate([F[:, 0], F[:, 1], F[:, 2]])
    tri = np.concatenate([np.arange(len(F))] * 3)
    key = np.lexsort(edge.T[::-1])
    edge, opp, tri = edge[key], opp[key], tri[key]
    same_next = np.all(edge[1:] == edge[:-1], axis=1)
    assert not np.any(same_next[1:] & same_next[:-1]), "edge in more than two triangles"
    first = np.flatnonzero(np.concatenate([[True], ~same_next]))
    count = np.diff(np.concatenate([first, [len(edge)]]))
    inner, hull = first[count == 2], first[count == 1]
    e = edge[inner]
    s1, fb1 = orient2_sign(P[e[:, 0]], P[e[:, 1]], P[opp[inner]])
    s2, fb2 = orient2_sign(P[e[:, 0]], P[e[:, 1]], P[opp[inner + 1]])
    assert np.all(s1 * s2 < 0), "triangles on the same side of a shared edge"
    T1 = F[tri[inner]]
    oo, _ = orient2_sign(P[T1[:, 0]], P[T1[:, 1]], P[T1[:, 2]])
    si, fb3 = incircle_sign(P[T1[:, 0]], P[T1[:, 1]], P[T1[:, 2]], P[opp[inner + 1]])
    assert np.all(si.astype(np.int64) * oo < 0), "not locally Delaunay (or cocircular)"
    h = edge[hull]
    side, _ = orient2_sign(P[h[:, 0]], P[h[:, 1]], P[opp[hull]])
    member = np.zeros((len(h), n), dtype=bool)
    member[np.arange(len(h))[:, None], h] = True
    sgn, fbh = orient2_sign(P[h[:, 0]][:, None], P[h[:, 1]][:, None], P[None, :, :], skip=member)
    bad = (sgn.astype(np.int64) * side.astype(np.int64)[:, None] < 0) | ((sgn == 0) & ~member)
    assert not np.any(bad), "hull edge is not a supporting line"
    assert len(np.unique(F)) == n, "point missing from the triangulation"
    E, _ = faces2d(F)
    assert n - len(E) + len(F) == 1, "Euler characteristic"
    return {"triangles": len(F), "hull_edges": len(hull), "exact_fallbacks": fb0 + fb1 + fb2 + fb3 + fbh}


def qhull_tris(P: np.ndarray) -> np.ndarray:
    """scipy's qhull Delaunay in the plane, canonicalised."""
    from scipy.spatial import Delaunay
    return canonical2(Delaunay(np.asarray(P, dtype=np.float64)).simplices)
