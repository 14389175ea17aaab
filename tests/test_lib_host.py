"""Host-side tests of the library (no GPU needed): exported symbols, argument
validation before any launch, and the host Delaunay against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_22432_amd as P
import synth
from oracle import delaunay as OD
from oracle import fps as OP
from paper_2509_22432_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "flood.h")).read()
    names = set(re.findall(r"\b(flood_[a-z0-9_]+)\s*\(", hdr))
    assert names == set(_lib.EXPORTED)
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n


def _fake_problem(k=4, B=1):
    pb = _lib.Problem()
    pb.B, pb.k, pb.landmarks_in_x = B, k, 0
    pb.X = pb.x_off_d = pb.Lxyz = pb.l_off_d = 0x1000
    off = (ctypes.c_int64 * 2)(0, 10)
    pb._keep = off
    pb.x_off = ctypes.cast(off, ctypes.POINTER(ctypes.c_int64))
    pb.l_off = ctypes.cast(off, ctypes.POINTER(ctypes.c_int64))
    zero = (ctypes.c_int64 * 2)(0, 0)
    pb._keep2 = zero
    for d in range(4):
        pb.s_off[d] = ctypes.cast(zero, ctypes.POINTER(ctypes.c_int64))
    return pb


@pytest.mark.parametrize("field,value,status", [("k", 0, _lib.EINVAL), ("k", 256, _lib.EUNSUPPORTED),
                                                ("B", 0, _lib.EINVAL), ("landmarks_in_x", 2, _lib.EINVAL)])
def test_filtration_rejects_bad_arguments(field, value, status):
    pb = _fake_problem()
    setattr(pb, field, value)
    out = _lib.Outputs()
    st = _lib.lib().flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), None, 0, None)
    assert st == status
    assert _lib.lib().flood_last_error().decode()


def test_filtration_rejects_small_workspace_and_bad_tuning():
    pb = _fake_problem()
    out = _lib.Outputs()
    for d in range(4):
        out.f[d] = out.win_x[d] = out.win_a[d] = 0x2000
    L = _lib.lib()
    assert L.flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), ctypes.c_void_p(0x3000), 16, None) == _lib.ENOMEM
    t = _lib.Tuning(100.0, 1, 4, 0, 0)
    assert L.flood_filtration(ctypes.byref(pb), ctypes.byref(t), ctypes.byref(out), None, 0, None) == _lib.EINVAL
    t = _lib.Tuning(1.0, 3, 4, 0, 0)
    assert L.flood_filtration(ctypes.byref(pb), ctypes.byref(t), ctypes.byref(out), None, 0, None) == _lib.EINVAL
    # the tile kernel runs at most four waves per block
    t = _lib.Tuning(1.0, 1, 5, 0, 0)
    assert L.flood_filtration(ctypes.byref(pb), ctypes.byref(t), ctypes.byref(out), None, 0, None) == _lib.EINVAL
    for bad in ((1.0, 1, 4, 33, 0), (1.0, 1, 4, -2, 0), (1.0, 1, 4, 0, 65), (1.0, 1, 4, 0, 1), (1.0, 1, 4, 0, 0, 3),
                (1.0, 1, 4, 0, 0, 16), (1.0, 1, 4, 0, 0, -1), (1.0, 1, 4, 0, 0, 0, 8), (1.0, 1, 4, 0, 0, 0, 48),
                (1.0, 1, 4, 0, 0, 0, -16)):
        t = _lib.Tuning(*bad)
        assert L.flood_filtration(ctypes.byref(pb), ctypes.byref(t), ctypes.byref(out), None, 0, None) == _lib.EINVAL


def test_fps_rejects_bad_arguments():
    L = _lib.lib()
    off = (ctypes.c_int64 * 2)(0, 10)
    n_lm = (ctypes.c_int32 * 1)(11)
    st = L.flood_fps(ctypes.c_void_p(0x1000), 1, off, ctypes.c_void_p(0x1000), n_lm, ctypes.c_void_p(0x1000), None,
                     ctypes.c_void_p(0x1000), None, None, 0, None)
    assert st == _lib.EINVAL
    n_lm[0] = 3
    st = L.flood_fps(ctypes.c_void_p(0x1000), 1, off, ctypes.c_void_p(0x1000), n_lm, ctypes.c_void_p(0x1000), None,
                     ctypes.c_void_p(0x1000), None, None, 0, None)
    assert st == _lib.ENOMEM
    assert L.flood_fps_workspace_size(1, off, n_lm) > 0


@pytest.mark.parametrize("cfg,n,L", [(1, None, 64), (2, 100_000, 600)])
def test_delaunay_bitexact(cfg, n, L):
    X = synth.config_cloud(cfg, n)
    idx, _ = OP.fps(X, L)
    Lx = X[idx]
    cx = P.delaunay(Lx)
    OD.certify(Lx, cx.T)
    assert np.array_equal(cx.T, OD.qhull_tets(Lx))
    E, F, te, tt = OD.faces(cx.T)
    assert np.array_equal(cx.E, E) and np.array_equal(cx.F, F)
    assert np.array_equal(cx.tri_edges, te) and np.array_equal(cx.tet_tris, tt)


@pytest.mark.parametrize("seed", range(5))
def test_delaunay_equals_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    Lx = rng.random((20 + 3 * seed, 3)).astype(np.float32)
    assert np.array_equal(P.delaunay(Lx).T, OD.brute_tets(Lx))


def test_delaunay_near_degenerate_uses_exact_fallback():
    # points on a sphere rounded to float32: many nearly cospherical 5-tuples
    rng = np.random.default_rng(3)
    d = rng.standard_normal((200, 3))
    Lx = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    cx = P.delaunay(Lx)
    OD.certify(Lx, cx.T)
    assert cx.fallbacks > 0


def test_delaunay_errors():
    with pytest.raises(P.FloodError) as e:
        P.delaunay(np.zeros((3, 3), np.float32))
    assert e.value.status == _lib.EDEGENERATE
    with pytest.raises(P.FloodError) as e:
        P.delaunay(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0.5, 0.5, 0]], np.float32))
    assert e.value.status == _lib.EDEGENERATE
    pts = np.random.default_rng(0).random((10, 3)).astype(np.float32)
    pts[5] = pts[2]
    with pytest.raises(P.FloodError) as e:
        P.delaunay(pts)
    assert e.value.status == _lib.EDEGENERATE
    bad = pts.copy()
    bad[0, 0] = np.nan
    with pytest.raises(P.FloodError) as e:
        P.delaunay(bad)
    assert e.value.status == _lib.EINVAL


def test_fps_undecided_landmarks_raise():
    # a cooperative FPS launch that gives up an exchange leaves -1 indices;
    # the binding turns them into an error instead of indexing row -1
    import torch
    from paper_2509_22432_amd import api
    api.check_landmarks(torch.tensor([0, 5, 3], dtype=torch.int32))
    with pytest.raises(P.FloodError) as e:
        api.check_landmarks(torch.tensor([0, 5, -1, -1], dtype=torch.int32))
    assert e.value.status == _lib.EHIP and "2 landmark" in str(e.value)


def test_noalloc_rejects_problems_beyond_the_static_scratch():
    # a problem whose workspace exceeds the 64 MiB static scratch is refused
    # before any launch (no GPU needed to see it)
    pb = _fake_problem(k=6)
    big = (ctypes.c_int64 * 2)(0, 5_000_000)
    pb._keep3 = big
    pb.x_off = ctypes.cast(big, ctypes.POINTER(ctypes.c_int64))
    out = _lib.Outputs()
    for d in range(4):
        out.f[d] = out.win_x[d] = out.win_a[d] = 0x2000
    L = _lib.lib()
    assert L.flood_filtration_workspace_size(ctypes.byref(pb), None) > 64 << 20
    st = L.flood_filtration_noalloc(ctypes.byref(pb), None, ctypes.byref(out), None)
    assert st == _lib.ENOMEM
    assert "static scratch" in L.flood_last_error().decode()


def test_sampling_mode_validation():
    L = _lib.lib()
    out = _lib.Outputs()
    for d in range(4):
        out.f[d] = out.win_x[d] = out.win_a[d] = 0x2000
    pb = _fake_problem()
    pb.sampling = 2
    assert L.flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), None, 0, None) == _lib.EINVAL
    pb = _fake_problem(k=70000)
    pb.sampling = _lib.SAMPLING_RANDOM
    assert L.flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), None, 0, None) == _lib.EUNSUPPORTED
    # random sets take up to 65536 samples per simplex (the grid stops at k = 255)
    pb = _fake_problem(k=1000)
    pb.sampling = _lib.SAMPLING_RANDOM
    assert L.flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), None, 0, None) == _lib.ENOMEM
    # win_w for some dimensions only (here vertices and edges exist)
    five = (ctypes.c_int64 * 2)(0, 5)
    pb._keep5 = five
    pb.s_off[1] = ctypes.cast(five, ctypes.POINTER(ctypes.c_int64))
    pb.simp[1] = pb.s_off_d[1] = 0x1000
    out.win_w[0] = 0x3000
    assert L.flood_filtration(ctypes.byref(pb), None, ctypes.byref(out), None, 0, None) == _lib.EINVAL
    assert "win_w" in L.flood_last_error().decode()
    # the backward of random sets needs the winners' weights
    out.win_w[0] = None
    g = (ctypes.c_void_p * 4)(0x4000, None, None, None)
    st = L.flood_filtration_backward(ctypes.byref(pb), ctypes.byref(out), g, ctypes.c_void_p(0x5000),
                                     ctypes.c_void_p(0x6000), None)
    assert st == _lib.EINVAL and "win_w" in L.flood_last_error().decode()


@pytest.mark.parametrize("seed", range(3))
def test_planar_delaunay_equals_brute_force_and_qhull(seed):
    rng = np.random.default_rng(400 + seed)
    Lx = rng.random((15 + 5 * seed, 2)).astype(np.float32)
    cx = P.delaunay(Lx)
    assert cx.T.shape == (0, 4) and cx.tet_tris.shape == (0, 4)
    assert np.array_equal(cx.F, OD.brute_tris(Lx))
    big = rng.random((3000, 2)).astype(np.float32)
    cb = P.delaunay(big)
    OD.certify2d(big, cb.F)
    assert np.array_equal(cb.F, OD.qhull_tris(big))
    E, te = OD.faces2d(cb.F)
    assert np.array_equal(cb.E, E) and np.array_equal(cb.tri_edges, te)


def test_planar_delaunay_errors_and_lift():
    with pytest.raises(P.FloodError) as e:
        P.delaunay(np.array([[0, 0], [1, 1], [2, 2], [3, 3]], np.float32))
    assert e.value.status == _lib.EDEGENERATE
    with pytest.raises(P.FloodError) as e:
        P.delaunay(np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32))  # cocircular square
    assert e.value.status == _lib.EDEGENERATE
    pts = np.random.default_rng(1).random((9, 2)).astype(np.float32)
    pts[4] = pts[7]
    with pytest.raises(P.FloodError) as e:
        P.delaunay(pts)
    assert e.value.status == _lib.EDEGENERATE
    lifted = P.lift_2d(np.ones((4, 2)))
    assert lifted.shape == (4, 3) and np.all(lifted[:, 2] == 0) and lifted.dtype == np.float32
