"""Ambient dimension 2 (Sec. 5.2 varies the ambient dimension): planar
clouds as [n, 3] rows with z = 0, landmarks by the same FPS recipe, the
planar Delaunay triangulation (vertices, edges, triangles) and the flooding
kernels unchanged.  Against the FP64 oracle: landmark indices bit for bit,
every simplex of a small cloud (grid and random sample sets), sampled
simplices of a 200k-point cloud (masked mode), and the planar Delaunay
certificate."""
import numpy as np
import pytest
import torch

import paper_2509_22432_amd as P
import synth
from oracle import delaunay as OD
from oracle import flood as OF
from oracle import fps as OP

from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _planar_run(X2, n_lm, k, sampling="grid", seed=0):
    X = P.lift_2d(X2)
    Xd = torch.from_numpy(X).to(dev())
    idx, _ = P.fps(Xd, n_lm)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    cx = P.delaunay(X2[idx])
    pb = P.problem_from_complexes(Xd, [0, len(X)], Xd[torch.from_numpy(idx).long().to(dev())].contiguous(),
                                  [0, n_lm], [cx], k, l_xidx=torch.from_numpy(idx.astype(np.int32)).to(dev()),
                                  sampling=sampling, seed=seed)
    run = P.filtration(pb)
    torch.cuda.synchronize()
    return X, idx, cx, [t.cpu().numpy() for t in run.f]


@pytest.mark.parametrize("sampling", ["grid", "random"])
def test_planar_all_simplices(sampling):
    X2 = synth.planar_cheese(3000, 6, seed=2101)
    k = 6 if sampling == "grid" else 24
    X, idx, cx, f = _planar_run(X2, 80, k, sampling, seed=77)
    oidx, _ = OP.fps(X, 80)
    assert np.array_equal(idx, oidx)
    OD.certify2d(X2[idx], cx.F)
    assert np.array_equal(cx.F, OD.qhull_tris(X2[idx]))
    assert len(cx.T) == 0
    cxo = dict(E=cx.E, F=cx.F, T=cx.T.reshape(0, 4), tri_edges=cx.tri_edges, tet_tris=cx.tet_tris.reshape(0, 4))
    if sampling == "grid":
        ref = OF.closure(OF.flood_all(X, X[idx], cxo, k, "brute"), cxo)
    else:
        ref = OF.closure(OF.flood_random_all(X, X[idx], cxo, k, 77, "brute"), cxo)
    diam = OF.diameter(X)
    err = [float(np.abs(f[d].astype(np.float64) - ref[d]).max()) if len(ref[d]) else 0.0 for d in range(3)]
    print("planar", sampling, "max|df|/diam per dim", [e / diam for e in err], flush=True)
    assert max(err) <= 1e-5 * diam
    assert np.all(f[0] == 0.0)
    assert np.all(f[0][cx.E].max(1) <= f[1])
    assert np.all(f[1][cx.tri_edges].max(1) <= f[2])
    assert len(f[3]) == 0


def test_planar_large_sampled_against_masked_oracle():
    X2 = synth.planar_cheese(200_000, 10, seed=2102)
    X, idx, cx, f = _planar_run(X2, 1000, 10)
    xs = OF.XSorted(X)
    diam = OF.diameter(X)
    rng = np.random.default_rng(9)
    for d, simp in ((1, cx.E), (2, cx.F)):
        pick = rng.choice(len(simp), 400, replace=False)
        ref, _, _ = OF.flood_dim(X, X[idx], simp[pick], d, 10, "masked", xs)
        err = np.abs(f[d][pick].astype(np.float64) - ref).max()
        print("planar 200k dim", d, "max|df|/diam", err / diam, flush=True)
        assert err <= 1e-5 * diam
