"""GPU parity for random sample sets (Thm. 5 with finite P_sigma inside conv
sigma; Lemma 9: points drawn uniformly): every simplex of dimension >= 1
owns m points drawn by the counter-based generator, and the closure over
faces makes f monotone.  The GPU draws its points with its own generator
code; the oracle with its own (FP64).

* every simplex of the torus cloud at m = 1, 16, 64 against the brute-force
  oracle with the closure, within 1e-5 * diam(X); monotonicity exact;
* the winners' weights equal the oracle's draws bit for bit (both sides
  produce exact multiples of 2^-24), x* attains f and is a nearest point;
* values identical across tunings; batched = plain;
* sampled simplices of the 1M-point cloud (and all their faces) against the
  masked oracle;
* the backward against the oracle's gradient, near ties given zero weight.
"""
import numpy as np
import pytest
import torch

import paper_2509_22432_amd as P
import synth
from oracle import flood as OF
from paper_2509_22432_amd import batch

from gpu_helpers import oracle_complex, run_single

pytestmark = pytest.mark.gpu
SIMP = {1: "E", 2: "F", 3: "T"}
SEED = 0x5EED1234ABCD


def _maxerr(res, ref):
    return [float(np.abs(res["out"]["f"][d].astype(np.float64) - ref[d]).max()) if len(ref[d]) else 0.0
            for d in range(4)]


@pytest.mark.parametrize("m", [1, 16, 64])
def test_random_config1_all_simplices(m):
    X = synth.config_cloud(1)
    res = run_single(X, 64, m, sampling="random", seed=SEED)
    cxo = oracle_complex(res["cx"])
    own = OF.flood_random_all(X, res["Lxyz"], cxo, m, SEED, "brute")
    ref = OF.closure(own, cxo)
    diam = OF.diameter(X)
    err = _maxerr(res, ref)
    print("random m", m, "max|df| per dim", err, "tol", 1e-5 * diam, flush=True)
    assert max(err) <= 1e-5 * diam
    f = res["out"]["f"]
    cx = res["cx"]
    assert np.all(f[0] == 0.0)
    assert np.all(f[0][cx.E].max(1) <= f[1])
    assert np.all(f[1][cx.tri_edges].max(1) <= f[2])
    assert np.all(f[2][cx.tet_tris].max(1) <= f[3])


def test_random_winners_and_weights():
    X = synth.config_cloud(1)
    m = 16
    res = run_single(X, 64, m, sampling="random", seed=SEED)
    cx, out = res["cx"], res["out"]
    L64, X64 = res["Lxyz"].astype(np.float64), X.astype(np.float64)
    diam = OF.diameter(X)
    for d in (1, 2, 3):
        simp = getattr(cx, SIMP[d])
        w = out["win_w"][d][:, :d + 1].astype(np.float64)
        wa = out["win_a"][d].astype(np.uint32)
        q = (wa & 0x0FFFFFFF).astype(np.int64)
        mask = (wa >> 28).astype(np.int64)
        own = mask == (1 << (d + 1)) - 1
        # own winners: the weights are the oracle generator's draws, exactly
        for j in np.flatnonzero(own)[:200]:
            ref_w = OF.random_weights(d, int(q[j]), int(j), SEED)
            assert np.array_equal(w[j].astype(np.float32), ref_w.astype(np.float32)), (d, j)
        # every winner: weights on the owner's vertices only, summing to 1
        for i in range(d + 1):
            assert np.all((w[:, i] > 0) <= ((mask >> i) & 1).astype(bool))
        assert np.allclose(w.sum(1), 1.0, atol=1e-6)
        sp = np.einsum("ni,nic->nc", w, L64[simp])
        dx = np.linalg.norm(sp - X64[out["win_x"][d]], axis=1)
        nn, _ = OF.nearest(X64, sp)
        assert np.abs(dx - out["f"][d]).max() <= 1e-5 * diam
        assert np.abs(nn - out["f"][d]).max() <= 1e-5 * diam


def test_random_tuning_invariance_and_batched_equals_plain():
    X = synth.config_cloud(2, 100_000)
    base = run_single(X, 400, 24, sampling="random", seed=7)
    for tu in ({"samples_per_lane": 2}, {"tile_shells": -1}, {"tile_shells": 2, "cells_per_point": 0.3},
               {"tile_lanes": 16}, {"tile_lanes": 32}):
        other = run_single(X, 400, 24, tuning=tu, sampling="random", seed=7)
        for d in range(4):
            for part in ("f", "win_x", "win_a", "win_w"):
                assert np.array_equal(base["out"][part][d], other["out"][part][d]), (tu, part, d)
    clouds, lms = synth.batched_clouds(5, seed=515, scale=0.1)
    pb, Ls, cxs = batch.prepare(clouds, lms, 12, sampling="random", seed=99)
    run = P.filtration(pb)
    torch.cuda.synchronize()
    for b, c in enumerate(clouds):
        single = run_single(c, lms[b], 12, sampling="random", seed=99)
        for d in range(4):
            so = pb.l_off if d == 0 else pb.s_off[d]
            sl = slice(int(so[b]), int(so[b + 1]))
            assert np.array_equal(run.f[d][sl].cpu().numpy(), single["out"]["f"][d]), (b, d)
            assert np.array_equal(run.win_w[d][sl].cpu().numpy(), single["out"]["win_w"][d]), (b, d)


def _face_rows(cx):
    """Row lookup of sorted vertex tuples per dimension."""
    return {1: {tuple(r): i for i, r in enumerate(cx.E.tolist())},
            2: {tuple(r): i for i, r in enumerate(cx.F.tolist())}}


def test_random_config2_sampled_against_masked_oracle():
    X = synth.config_cloud(2)
    m = 64
    res = run_single(X, 2000, m, sampling="random", seed=SEED)
    cx = res["cx"]
    xs = OF.XSorted(X)
    diam = OF.diameter(X)
    rows = _face_rows(cx)
    rng = np.random.default_rng(3)
    from itertools import combinations
    for d in (1, 2, 3):
        simp = getattr(cx, SIMP[d])
        pick = rng.choice(len(simp), 200, replace=False)
        # f(sigma) = max over the faces of dimension >= 1 of their own value
        # (vertex values are 0: the landmarks are points of X)
        best = np.zeros(len(pick))
        for e in range(1, d + 1):
            faces, frows = [], []
            for j in pick:
                for sub in combinations(simp[j].tolist(), e + 1):
                    faces.append(sub)
                    frows.append(j if e == d else rows[e][sub])
            own, _, _ = OF.flood_random_dim(X, res["Lxyz"], np.array(faces), e, m, SEED, rows=np.array(frows),
                                            mode="masked", xsorted=xs)
            nf = len(faces) // len(pick)
            best = np.maximum(best, own.reshape(len(pick), nf).max(1))
        err = np.abs(res["out"]["f"][d][pick].astype(np.float64) - best).max()
        print("random config 2 dim", d, "max|df|/diam", err / diam, flush=True)
        assert err <= 1e-5 * diam


def _random_tie_gaps(X, L, cx, m, seed):
    """Per simplex: the gap between the two largest sample values over the
    whole closure (own samples and every face's), and between the two
    nearest points of the winning sample (brute force, FP64)."""
    from itertools import combinations
    X64 = X.astype(np.float64)
    rows = {1: {tuple(r): i for i, r in enumerate(cx["E"].tolist())},
            2: {tuple(r): i for i, r in enumerate(cx["F"].tolist())},
            3: {tuple(r): i for i, r in enumerate(cx["T"].tolist())}}
    cache = {}

    def samples(face):
        e = len(face) - 1
        if face not in cache:
            if e == 0:
                P_ = L[list(face)].astype(np.float64)
            else:
                r = rows[e][face]
                W = np.stack([OF.random_weights(e, q, r, seed) for q in range(m)])
                P_ = W @ L[list(face)].astype(np.float64)
            dist = np.sqrt(((P_[:, None, :] - X64[None]) ** 2).sum(-1))
            part = np.sort(dist, axis=1)[:, :2]
            cache[face] = part
        return cache[face]

    gaps = {}
    for d in (1, 2, 3):
        simp = cx[SIMP[d]]
        g = np.empty(len(simp))
        for j, s in enumerate(simp.tolist()):
            parts = np.concatenate([samples(sub) for e in range(d + 1) for sub in combinations(s, e + 1)])
            nn = parts[:, 0]
            order = np.argsort(nn)
            g1 = nn[order[-1]] - nn[order[-2]]
            b = order[-1]
            g[j] = min(g1, parts[b, 1] - parts[b, 0])
        gaps[d] = g
    return gaps


def test_random_backward_matches_oracle_gradient():
    X = synth.differentiable_clouds(1, 2500, seed=5)[0]
    m = 12
    res = run_single(X, 40, m, sampling="random", seed=SEED)
    cx = oracle_complex(res["cx"])
    Lx = res["Lxyz"]
    diam = OF.diameter(X)
    vals = OF.flood_random_all(X, Lx, cx, m, SEED, "brute")
    gaps = _random_tie_gaps(X, Lx, cx, m, SEED)
    rng = np.random.default_rng(2)
    w = {0: rng.random(len(vals[0][0]))}
    for d in (1, 2, 3):
        w[d] = rng.random(len(vals[d][0]))
        w[d][gaps[d] <= 1e-4 * diam] = 0.0
    gX_ref, gL_ref = OF.random_gradient(X, Lx, cx, vals, m, SEED, w)
    run = res["run"]
    gX = torch.zeros_like(run.pb.X)
    gL = torch.zeros_like(run.pb.Lxyz)
    run.backward([torch.from_numpy(w[d].astype(np.float32)).to(gX.device) for d in range(4)], gX, gL)
    torch.cuda.synchronize()
    gX, gL = gX.cpu().numpy(), gL.cpu().numpy()
    print("random backward: max |dgX|", np.abs(gX - gX_ref).max(), "max |dgL|", np.abs(gL - gL_ref).max(),
          "weighted", [int((w[d] > 0).sum()) for d in range(4)], flush=True)
    assert np.abs(gX - gX_ref).max() <= 1e-4 * (1 + np.abs(gX_ref).max())
    assert np.abs(gL - gL_ref).max() <= 1e-4 * (1 + np.abs(gL_ref).max())
