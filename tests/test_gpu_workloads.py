"""GPU parity at the workload shapes: persistence diagrams, batched clouds
(FP32 GPU vs FP64 oracle, per simplex dimension) and the gradient at the
differentiable workload's shape."""
import numpy as np
import pytest
import torch

import paper_2509_22432_amd as P
import synth
from oracle import flood as OF
from oracle import ph as OPH
from paper_2509_22432_amd import batch

from gpu_helpers import oracle_complex, run_single

pytestmark = pytest.mark.gpu
SIMP = {1: "E", 2: "F", 3: "T"}


def test_persistence_diagrams_match():
    X = synth.config_cloud(1)
    k = 4
    res = run_single(X, 64, k)
    cx = oracle_complex(res["cx"])
    ref = OF.closure(OF.flood_all(X, res["Lxyz"], cx, k), cx)
    gpu = {d: res["out"]["f"][d].astype(np.float64) for d in range(4)}
    tol = 1e-5 * OF.diameter(X)
    dg_ref = OPH.diagrams(cx, ref, maxdim=2)
    dg_gpu = OPH.diagrams(cx, gpu, maxdim=2)
    for p in range(3):
        print("dim", p, "finite pairs", len(dg_ref[p][0]), len(dg_gpu[p][0]), "essential", len(dg_ref[p][1]))
        # near-zero persistence pairs may appear on one side only: the
        # matching lets them go to the diagonal within tol
        assert OPH.bottleneck_leq(dg_ref[p], dg_gpu[p], tol)
    # the library's persistence step on the GPU values: the same diagrams as
    # the oracle's reduction on those values, exactly
    lib_dg = P.persistence(res["cx"], [res["out"]["f"][d] for d in range(4)])
    for p in range(3):
        fin = np.isfinite(lib_dg[p]["death"])
        got = np.stack([lib_dg[p]["birth"][fin], lib_dg[p]["death"][fin]], 1).astype(np.float64)
        want = dg_gpu[p][0].reshape(-1, 2)
        srt = lambda a: a[np.lexsort((a[:, 1], a[:, 0]))]
        assert np.array_equal(srt(got), srt(want)), p
        assert np.array_equal(np.sort(lib_dg[p]["birth"][~fin].astype(np.float64)), np.sort(dg_gpu[p][1])), p


def test_batched_clouds_fp32_vs_fp64_per_dim():
    clouds, lms = synth.batched_clouds(24, seed=777, scale=0.25)
    k = 6
    pb, Ls, cxs = batch.prepare(clouds, lms, k)
    run = P.filtration(pb)
    torch.cuda.synchronize()
    f = [t.cpu().numpy().astype(np.float64) for t in run.f]
    rng = np.random.default_rng(3)
    worst = np.zeros(4)
    for b in range(len(clouds)):
        X = clouds[b]
        tol = 1e-5 * OF.diameter(X)
        xs = OF.XSorted(X)
        for d in range(4):
            simp = np.arange(cxs[b].L).reshape(-1, 1) if d == 0 else getattr(cxs[b], SIMP[d])
            off = int(pb.l_off[b]) if d == 0 else int(pb.s_off[d][b])
            pick = rng.choice(len(simp), min(60, len(simp)), replace=False)
            ref, _, _ = OF.flood_dim(X, Ls[b], simp[pick], d, k, "masked", xs)
            # the value is the closure of the full grid; the oracle's full grid
            # already includes every face sample
            err = np.abs(f[d][off + pick] - ref).max()
            worst[d] = max(worst[d], err / tol)
            assert err <= tol, (b, d, err, tol)
    print("max |df| / tol per dimension over the sampled clouds:", worst)


def test_gradient_at_differentiable_shape():
    X = synth.differentiable_clouds(1, 100_000, seed=1005)[0]
    k = 6
    res = run_single(X, 512, k)
    cxo = oracle_complex(res["cx"])
    Lx = res["Lxyz"]
    diam = OF.diameter(X)
    xs = OF.XSorted(X)
    rng = np.random.default_rng(4)
    w = {0: rng.random(512)}  # f = 0 on vertices: u = 0 on both sides
    vals = {0: OF.flood_dim(X, Lx, np.arange(512).reshape(-1, 1), 0, k, "masked", xs)}
    for d in (1, 2, 3):
        simp = cxo[SIMP[d]]
        w[d] = np.zeros(len(simp))
        pick = rng.choice(len(simp), min(1500, len(simp)), replace=False)
        fv, wa, wx, gs, gx = OF.flood_dim(X, Lx, simp[pick], d, k, "masked", xs, gaps=True)
        full_f = np.zeros(len(simp))
        full_wa = np.zeros((len(simp), 4), np.int32)
        full_wx = np.zeros(len(simp), np.int32)
        full_f[pick], full_wa[pick], full_wx[pick] = fv, wa, wx
        ok = (gs > 1e-4 * diam) & (gx > 1e-4 * diam)
        w[d][pick[ok]] = rng.random(int(ok.sum()))
        # with the ties excluded, the oracle's first attaining sample and the
        # GPU's winner (own interior sample or inherited from a facet) are
        # the same grid point, so the two gradients agree term by term
        vals[d] = (full_f, full_wa, full_wx)
    gX_ref, gL_ref = OF.gradient(X, Lx, cxo, vals, k, w)
    run = res["run"]
    gX = torch.zeros_like(run.pb.X)
    gL = torch.zeros_like(run.pb.Lxyz)
    run.backward([torch.from_numpy(w[d].astype(np.float32)).to(gX.device) for d in range(4)], gX, gL)
    torch.cuda.synchronize()
    gX, gL = gX.cpu().numpy(), gL.cpu().numpy()
    print("max |dgX|", np.abs(gX - gX_ref).max(), "max |dgL|", np.abs(gL - gL_ref).max())
    assert np.abs(gX - gX_ref).max() <= 1e-4 * (1 + np.abs(gX_ref).max())
    assert np.abs(gL - gL_ref).max() <= 1e-4 * (1 + np.abs(gL_ref).max())
