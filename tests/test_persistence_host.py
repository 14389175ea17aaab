"""The library's persistence step (host C++) against the oracle's reduction.

Both order simplices by (f, dimension, vertex tuple), so the diagrams must
agree exactly: the same multiset of (birth, death) values per dimension and
the same essential births.  The oracle's reduction is pinned in
test_oracle_ph.py (textbook complexes, rank-invariant persistence, circle
diagrams).
"""
import numpy as np
import pytest

import paper_2509_22432_amd as P
import synth
from oracle import flood as OF
from oracle import fps as OP
from oracle import ph
from paper_2509_22432_amd import _lib


def _oracle_cx(cx):
    return {"L": cx.L, "E": cx.E, "F": cx.F, "T": cx.T}


def _assert_same(dg, ref):
    for p in range(3):
        fin_ref, ess_ref = ref[p]
        fin = np.isfinite(dg[p]["death"])
        got = np.stack([dg[p]["birth"][fin], dg[p]["death"][fin]], 1).astype(np.float64)
        key = lambda a: a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a.reshape(0, 2)
        assert np.array_equal(key(got), key(fin_ref.reshape(-1, 2))), p
        assert np.array_equal(np.sort(dg[p]["birth"][~fin].astype(np.float64)), np.sort(ess_ref)), p


def _monotone_values(cx, rng, levels=None):
    """Random filtration values with f(face) <= f(coface); `levels` quantises
    them so that exact ties are frequent."""
    draw = (lambda n: rng.integers(0, levels, n).astype(np.float32)) if levels else \
        (lambda n: rng.random(n).astype(np.float32))
    f0 = draw(cx.L)
    f1 = np.maximum(draw(len(cx.E)), np.maximum(f0[cx.E[:, 0]], f0[cx.E[:, 1]]))
    f2 = np.maximum(draw(len(cx.F)), f1[cx.tri_edges].max(1))
    f3 = np.maximum(draw(len(cx.T)), f2[cx.tet_tris].max(1)) if len(cx.T) else np.zeros(0, np.float32)
    return [f0, f1, f2, f3]


@pytest.mark.parametrize("seed,L,levels", [(0, 40, None), (1, 80, None), (2, 60, 4), (3, 120, 2)])
def test_random_filtrations_match_oracle(seed, L, levels):
    rng = np.random.default_rng(seed)
    Lxyz = rng.random((L, 3)).astype(np.float32)
    cx = P.delaunay(Lxyz)
    f = _monotone_values(cx, rng, levels)
    dg = P.persistence(cx, f)
    ref = ph.diagrams(_oracle_cx(cx), {d: f[d] for d in range(4)}, maxdim=2)
    _assert_same(dg, ref)
    # a Delaunay complex is a 3-ball: one component, no cycles or voids left
    assert [int(np.isinf(dg[p]["death"]).sum()) for p in range(3)] == [1, 0, 0]


def test_flood_values_of_the_torus_match_oracle():
    X = synth.config_cloud(1)
    idx, _ = OP.fps(X, 64)
    Lxyz = X[idx]
    cx = P.delaunay(Lxyz)
    ocx = _oracle_cx(cx)
    fr = OF.flood_all(X, Lxyz, {"L": cx.L, "E": cx.E, "F": cx.F, "T": cx.T}, 4, "brute")
    f = [np.asarray(fr[d][0], dtype=np.float32) for d in range(4)]
    # the float32 values keep the closure exactly (rounding is monotone)
    dg = P.persistence(cx, f)
    _assert_same(dg, ph.diagrams(ocx, {d: f[d] for d in range(4)}, maxdim=2))
    # rows point at simplices that carry the reported values
    E = dg[1]
    fin = np.isfinite(E["death"])
    assert np.array_equal(f[1][E["birth_row"]], E["birth"])
    assert np.array_equal(f[2][E["death_row"][fin]], E["death"][fin])


def _raw(n, E, te, tt, f):
    import ctypes
    L = _lib.lib()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    arrs = [np.ascontiguousarray(x, dtype=np.float32) for x in f]
    h = ctypes.c_void_p()
    st = L.flood_persistence((ctypes.c_int64 * 4)(*n), vp(E), vp(te), vp(tt),
                             (ctypes.c_void_p * 4)(*[vp(a) if len(a) else None for a in arrs]), ctypes.byref(h))
    return st, h, L


def test_textbook_complexes():
    # hollow tetrahedron at one level: one component and one void
    E = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]], np.int32)
    # triangles (012, 013, 023, 123): facet i omits vertex i
    te = np.array([[3, 1, 0], [4, 2, 0], [5, 2, 1], [5, 4, 3]], np.int32)
    st, h, L = _raw([4, 6, 4, 0], E, te, None, [np.zeros(4), np.zeros(6), np.zeros(4), np.zeros(0)])
    assert st == _lib.OK
    import ctypes
    cnt = (ctypes.c_int64 * 3)()
    assert L.flood_diagram_counts(h, cnt) == _lib.OK
    assert list(cnt) == [1, 0, 1]
    L.flood_diagram_free(h)
    # triangle boundary: one component, one loop born at the last edge
    st, h, L = _raw([3, 3, 0, 0], E[[0, 1, 3]], None, None,
                    [np.zeros(3), np.array([1, 2, 3]), np.zeros(0), np.zeros(0)])
    assert st == _lib.OK
    assert L.flood_diagram_counts(h, cnt) == _lib.OK
    assert list(cnt) == [3, 1, 0]  # two finite H0 pairs (0,1), (0,2) and one essential each
    b = np.zeros(1, np.float32)
    assert L.flood_diagram_export(h, 1, b.ctypes.data_as(ctypes.c_void_p), None, None, None) == _lib.OK
    assert b[0] == 3.0
    L.flood_diagram_free(h)


def test_rejects_invalid_filtrations():
    E = np.array([[0, 1], [0, 2], [1, 2]], np.int32)
    te = np.array([[2, 1, 0]], np.int32)
    ok = [np.zeros(3), np.ones(3), np.full(1, 2.0), np.zeros(0)]
    assert _raw([3, 3, 1, 0], E, te, None, ok)[0] == _lib.OK
    bad = [np.zeros(3), np.ones(3), np.full(1, 0.5), np.zeros(0)]  # triangle below its edges
    assert _raw([3, 3, 1, 0], E, te, None, bad)[0] == _lib.EINVAL
    nan = [np.zeros(3), np.array([1, np.nan, 1]), np.full(1, 2.0), np.zeros(0)]
    assert _raw([3, 3, 1, 0], E, te, None, nan)[0] == _lib.EINVAL
    far = np.array([[0, 1], [0, 7], [1, 2]], np.int32)  # vertex 7 does not exist
    assert _raw([3, 3, 1, 0], far, te, None, ok)[0] == _lib.EINVAL
    assert _raw([3, 3, 1, 0], None, te, None, ok)[0] == _lib.EINVAL
    assert _lib.lib().flood_last_error().decode()
