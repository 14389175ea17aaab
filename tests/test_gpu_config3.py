"""GPU parity at the benchmark's full size: N = 10,000,000 points on 20 noisy
primitive surfaces, L = 10,000 farthest-point landmarks, k = 8, in the launch
configuration the benchmark times (default tuning).

* Del(L) is certified (Delaunay's lemma: every interior triangle locally
  Delaunay, hull triangles supporting, Euler characteristic 1) and equal to
  qhull's, here and for the 1M-point cloud's 2,000 landmarks.
* f is compared element by element with the FP64 oracle (masked mode,
  exact by Lemma 7 since L is a subset of X) on 2,000 seeded random
  simplices per dimension, at 1e-5 * diam(X); the largest |df| / diam(X)
  per dimension is printed.
* Properties that hold at any size are checked on every simplex: vertex
  values are 0 (landmarks are points of X) and f(face) <= f(coface).
"""
import numpy as np
import pytest
import torch

import paper_2509_22432_amd as P
import synth
from oracle import delaunay as OD
from oracle import flood as OF

from gpu_helpers import dev

pytestmark = pytest.mark.gpu
SIMP = {1: "E", 2: "F", 3: "T"}
N_CHECK = 2000


@pytest.fixture(scope="module")
def cfg3():
    X = synth.config_cloud(3)
    print("config 3: N", len(X), flush=True)
    Xd = torch.from_numpy(X).to(dev())
    idx, _ = P.fps(Xd, 10_000)
    torch.cuda.synchronize()
    Lxyz = X[idx.cpu().numpy()]
    cx = P.delaunay(Lxyz)
    pb = P.problem_from_complexes(Xd, [0, len(X)], Xd[idx.long()].contiguous(), [0, len(Lxyz)], [cx], 8,
                                  l_xidx=idx.clone())
    run = P.filtration(pb)
    torch.cuda.synchronize()
    f = [t.cpu().numpy() for t in run.f]
    print("config 3: counts", cx.counts(), "evals", int(run.evals.item()), flush=True)
    del run, pb
    torch.cuda.empty_cache()
    return dict(X=X, Lxyz=Lxyz, cx=cx, f=f, diam=OF.diameter(X), xs=OF.XSorted(X))


def test_config3_delaunay_certified(cfg3):
    cx, L = cfg3["cx"], cfg3["Lxyz"]
    info = OD.certify(L, cx.T)
    print("certificate", info, flush=True)
    assert np.array_equal(cx.T, OD.qhull_tets(L))
    E, F, te, tt = OD.faces(cx.T)
    assert np.array_equal(cx.E, E) and np.array_equal(cx.F, F)
    assert np.array_equal(cx.tri_edges, te) and np.array_equal(cx.tet_tris, tt)


def test_config2_delaunay_certified():
    X = synth.config_cloud(2)
    idx, _ = P.fps(torch.from_numpy(X).to(dev()), 2000)
    L = X[idx.cpu().numpy()]
    cx = P.delaunay(L)
    print("config 2 certificate", OD.certify(L, cx.T), flush=True)
    assert np.array_equal(cx.T, OD.qhull_tets(L))
    E, F, te, tt = OD.faces(cx.T)
    assert np.array_equal(cx.E, E) and np.array_equal(cx.F, F)


def test_config3_every_simplex_properties(cfg3):
    f, cx = cfg3["f"], cfg3["cx"]
    assert np.all(f[0] == 0.0)
    assert np.all(f[0][cx.E].max(1) <= f[1])
    assert np.all(f[1][cx.tri_edges].max(1) <= f[2])
    assert np.all(f[2][cx.tet_tris].max(1) <= f[3])
    assert all(np.all(np.isfinite(v)) for v in f)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_config3_sampled_against_masked_oracle(cfg3, d):
    simp = getattr(cfg3["cx"], SIMP[d])
    rng = np.random.default_rng(100 + d)
    pick = np.sort(rng.choice(len(simp), N_CHECK, replace=False))
    ref, _, _ = OF.flood_dim(cfg3["X"], cfg3["Lxyz"], simp[pick], d, 8, "masked", cfg3["xs"])
    err = np.abs(cfg3["f"][d][pick].astype(np.float64) - ref)
    print("config 3 dim %d: max|df|/diam = %.3e over %d simplices (tol 1e-5)" % (d, err.max() / cfg3["diam"],
                                                                                  len(pick)), flush=True)
    assert err.max() <= 1e-5 * cfg3["diam"]
