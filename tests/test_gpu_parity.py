"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance for flood values: 1e-5 * diam(X) (FP32 GPU vs FP64 oracle).
Landmark indices and Delaunay simplices: bit-exact.
"""
import numpy as np
import pytest
import torch

import paper_2509_22432_amd as P
import synth
from oracle import delaunay as OD
from oracle import flood as OF
from oracle import fps as OP

from gpu_helpers import dev, oracle_complex, run_single, unpack

pytestmark = pytest.mark.gpu
SIMP = {1: "E", 2: "F", 3: "T"}


def _maxerr_per_dim(res, ref):
    return [float(np.abs(res["out"]["f"][d].astype(np.float64) - ref[d][0]).max()) if len(ref[d][0]) else 0.0
            for d in range(4)]


# ---------------------------------------------------------------- landmarks

@pytest.mark.parametrize("cfg,n,L", [(1, None, 64), (2, 12_000, 300), (2, 20_000, 500), (2, 200_000, 700),
                                     (2, None, 2000), (3, None, 10_000)])
def test_fps_bitexact(cfg, n, L):
    X = synth.config_cloud(cfg, n)
    print("fps parity cfg", cfg, "N", len(X), "L", L, flush=True)
    idx, rad = P.fps(torch.from_numpy(X).to(dev()), L)
    torch.cuda.synchronize()
    oidx, orad = OP.fps(X, L)
    assert np.array_equal(idx.cpu().numpy(), oidx)
    assert np.array_equal(rad.cpu().numpy(), orad)


def test_fps_lattice_ties_and_start():
    # 531441 lattice points take the cooperative path; exact ties are decided
    # by the lowest point index, and the first landmark is not point 0
    X = synth.lattice_points(81)
    print("fps lattice N", len(X), flush=True)
    for start, L in ((12345, 600), (0, 64)):
        idx, rad = P.fps(torch.from_numpy(X).to(dev()), L, start=start)
        torch.cuda.synchronize()
        oidx, orad = OP.fps(X, L, start=start)
        assert idx.cpu().numpy()[0] == start
        assert np.array_equal(idx.cpu().numpy(), oidx)
        assert np.array_equal(rad.cpu().numpy(), orad)


@pytest.mark.parametrize("n_clouds", [7, 12])
def test_fps_batched_bitexact(n_clouds):
    # 7 clouds: those of at least 2^12 points take cooperative launches, the
    # others one workgroup each, in the same call; 12 clouds: all of them
    # one workgroup each
    clouds, lms = synth.batched_clouds(n_clouds, seed=4242, scale=0.2)
    x_off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])])
    Xd = torch.from_numpy(np.concatenate(clouds)).to(dev())
    idx, rad = P.fps_batched(Xd, x_off, lms)
    torch.cuda.synchronize()
    idx, rad = idx.cpu().numpy(), rad.cpu().numpy()
    o = 0
    for c, l in zip(clouds, lms):
        oi, orad = OP.fps(c, l)
        assert np.array_equal(idx[o:o + l], oi)
        assert np.array_equal(rad[o:o + l], orad)
        o += l


def test_fps_circle_stages():
    N = 1024
    X = synth.circle_points(N)
    idx, _ = P.fps(torch.from_numpy(X).to(dev()), 64)
    idx = idx.cpu().numpy()
    for s in range(1, 7):
        assert set(idx[: 2 ** s].tolist()) == set(range(0, N, N // 2 ** s))


# ------------------------------------------------------------ flood values

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8])
def test_flood_config1_all_simplices(k):
    X = synth.config_cloud(1)
    res = run_single(X, 64, k)
    ref = OF.flood_all(X, res["Lxyz"], oracle_complex(res["cx"]), k, "brute")
    diam = OF.diameter(X)
    err = _maxerr_per_dim(res, ref)
    print("k", k, "max|df| per dim", err, "tol", 1e-5 * diam, "evals", res["out"]["evals"])
    assert max(err) <= 1e-5 * diam
    f = res["out"]["f"]
    assert np.all(f[0] == 0.0)   # landmarks are points of X
    cx = res["cx"]
    assert np.all(f[0][cx.E].max(1) <= f[1])
    assert np.all(f[1][cx.tri_edges].max(1) <= f[2])
    assert np.all(f[2][cx.tet_tris].max(1) <= f[3])


def test_delaunay_bitexact_vs_oracle():
    X = synth.config_cloud(2, 300_000)
    idx, _ = P.fps(torch.from_numpy(X).to(dev()), 1500)
    L = X[idx.cpu().numpy()]
    cx = P.delaunay(L)
    OD.certify(L, cx.T)
    assert np.array_equal(cx.T, OD.qhull_tets(L))
    E, F, te, tt = OD.faces(cx.T)
    assert np.array_equal(cx.E, E) and np.array_equal(cx.F, F)
    assert np.array_equal(cx.tri_edges, te) and np.array_equal(cx.tet_tris, tt)


def test_tuning_invariance_and_determinism():
    X = synth.config_cloud(2, 100_000)
    base = run_single(X, 400, 6)
    again = run_single(X, 400, 6)
    for d in range(4):
        assert np.array_equal(base["out"]["f"][d], again["out"]["f"][d])
        assert np.array_equal(base["out"]["win_x"][d], again["out"]["win_x"][d])
        assert np.array_equal(base["out"]["win_a"][d], again["out"]["win_a"][d])
    # the number of evaluations may differ: the running max M that retires
    # samples is read while other tiles are still raising it
    for tu in ({"samples_per_lane": 2}, {"samples_per_lane": 4}, {"cells_per_point": 0.2},
               {"cells_per_point": 6.0, "waves_per_block": 1}, {"tile_shells": -1}, {"tile_shells": 1},
            {"tile_shells": 4, "samples_per_lane": 2}, {"tile_shells": 2}, {"tile_shells": 16},
            {"tile_shells": 32, "tile_extent": 64}, {"tile_lanes": 32}, {"tile_lanes": 16},
            {"tile_lanes": 16, "tile_shells": 2}, {"tile_lanes": 64}, {"tile_lanes": 16, "samples_per_lane": 2}):
        other = run_single(X, 400, 6, tuning=tu)
        for d in range(4):
            assert np.array_equal(base["out"]["f"][d], other["out"]["f"][d]), (tu, d)
            assert np.array_equal(base["out"]["win_x"][d], other["out"]["win_x"][d]), (tu, d)
            assert np.array_equal(base["out"]["win_a"][d], other["out"]["win_a"][d]), (tu, d)


def test_winners_attain_values():
    X = synth.config_cloud(1)
    k = 4
    res = run_single(X, 64, k)
    cx, out = res["cx"], res["out"]
    L64, X64 = res["Lxyz"].astype(np.float64), X.astype(np.float64)
    diam = OF.diameter(X)
    for d in (1, 2, 3):
        simp = getattr(cx, SIMP[d])
        a = unpack(out["win_a"][d], d)
        assert np.all(a.sum(1) == k)
        sp = OF.winner_points(L64, simp, a, k)
        dx = np.linalg.norm(sp - X64[out["win_x"][d]], axis=1)
        nn, _ = OF.nearest(X64, sp)
        assert np.abs(dx - out["f"][d]).max() <= 1e-5 * diam
        assert np.abs(nn - out["f"][d]).max() <= 1e-5 * diam


def test_landmarks_not_in_x():
    X = synth.config_cloud(1)
    rng = np.random.default_rng(5)
    Lx = (rng.random((40, 3)) * np.ptp(X, 0) + X.min(0)).astype(np.float32)
    k = 4
    res = run_single(X, None, k, landmarks=Lx)
    ref = OF.flood_all(X, Lx, oracle_complex(res["cx"]), k, "brute")
    assert max(_maxerr_per_dim(res, ref)) <= 1e-5 * OF.diameter(X)
    assert np.all(res["out"]["f"][0] > 0)


def test_batched_equals_plain():
    clouds, lms = synth.batched_clouds(6, seed=99, scale=0.1)
    k = 6
    x_off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])])
    Xd = torch.from_numpy(np.concatenate(clouds)).to(dev())
    idx, _ = P.fps_batched(Xd, x_off, lms)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy()
    l_off = np.concatenate([[0], np.cumsum(lms)])
    cxs, Ls, gidx = [], [], []
    for b, c in enumerate(clouds):
        li = idx[l_off[b]:l_off[b + 1]]
        Ls.append(c[li])
        cxs.append(P.delaunay(c[li]))
        gidx.append(li + x_off[b])
    Ld = torch.from_numpy(np.concatenate(Ls)).to(dev())
    gi = torch.from_numpy(np.concatenate(gidx).astype(np.int32)).to(dev())
    pb = P.problem_from_complexes(Xd, x_off, Ld, l_off, cxs, k, l_xidx=gi)
    run = P.filtration(pb)
    torch.cuda.synchronize()
    for b, c in enumerate(clouds):
        single = run_single(c, lms[b], k)
        for d in range(4):
            so = pb.l_off if d == 0 else pb.s_off[d]
            sl = slice(int(so[b]), int(so[b + 1]))
            assert np.array_equal(run.f[d][sl].cpu().numpy(), single["out"]["f"][d]), (b, d)
            wx = run.win_x[d][sl].cpu().numpy() - x_off[b]
            assert np.array_equal(wx, single["out"]["win_x"][d]), (b, d)


@pytest.mark.parametrize("k", [6, 255])
def test_single_tetrahedron_extremes(k):
    rng = np.random.default_rng(12)
    X = rng.random((60, 3)).astype(np.float32)
    res = run_single(X, 4, k)
    assert res["cx"].counts() == (4, 6, 4, 1)
    ref = OF.flood_all(X, res["Lxyz"], oracle_complex(res["cx"]), k, "brute")
    assert max(_maxerr_per_dim(res, ref)) <= 1e-5 * OF.diameter(X)


def test_config2_sampled_against_masked_oracle():
    X = synth.config_cloud(2)
    k = 10
    res = run_single(X, 2000, k)
    print("config 2 counts", res["cx"].counts(), "evals", res["out"]["evals"], flush=True)
    xsorted = OF.XSorted(X)
    rng = np.random.default_rng(0)
    diam = OF.diameter(X)
    for d in (1, 2, 3):
        simp = getattr(res["cx"], SIMP[d])
        pick = np.sort(rng.choice(len(simp), 150, replace=False))
        ref, _, _ = OF.flood_dim(X, res["Lxyz"], simp[pick], d, k, "masked", xsorted)
        err = np.abs(res["out"]["f"][d][pick].astype(np.float64) - ref).max()
        print("dim", d, "max|df| on 150 sampled", err)
        assert err <= 1e-5 * diam


def test_base_tuning_against_oracle_and_metamorphic():
    # the default-tuning run the invariance test compares against, checked
    # against the masked oracle; then two transformations that must leave
    # the values exactly as they are: a permutation of the rows of X (the
    # landmarks kept as the same points), and scaling every coordinate by 2
    # (every correctly rounded operation commutes with it, so f doubles bit
    # for bit and the landmark indices do not change)
    X = synth.config_cloud(2, 100_000)
    k = 6
    base = run_single(X, 400, k)
    xs = OF.XSorted(X)
    diam = OF.diameter(X)
    rng = np.random.default_rng(21)
    for d in (1, 2, 3):
        simp = getattr(base["cx"], SIMP[d])
        pick = rng.choice(len(simp), 300, replace=False)
        ref, _, _ = OF.flood_dim(X, base["Lxyz"], simp[pick], d, k, "masked", xs)
        assert np.abs(base["out"]["f"][d][pick].astype(np.float64) - ref).max() <= 1e-5 * diam
    perm = rng.permutation(len(X))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(X))
    Xp = np.ascontiguousarray(X[perm])
    Xd = torch.from_numpy(Xp).to(dev())
    lx = torch.from_numpy(inv[base["idx"]].astype(np.int32)).to(dev())
    Ld = torch.from_numpy(base["Lxyz"]).to(dev())
    pb = P.problem_from_complexes(Xd, [0, len(X)], Ld, [0, len(base["Lxyz"])], [base["cx"]], k, l_xidx=lx)
    run = P.filtration(pb)
    torch.cuda.synchronize()
    for d in range(4):
        assert np.array_equal(run.f[d].cpu().numpy(), base["out"]["f"][d]), d
        assert np.array_equal(run.win_a[d].cpu().numpy().view(np.uint32), base["out"]["win_a"][d]), d
        # x* is the same point (exact ties between distinct points, where the
        # lowest row would decide, do not occur in these noisy clouds)
        assert np.array_equal(Xp[run.win_x[d].cpu().numpy()], X[base["out"]["win_x"][d]]), d
    scaled = run_single(np.ascontiguousarray(X * np.float32(2)), 400, k)
    assert np.array_equal(scaled["idx"], base["idx"])
    for d in range(4):
        assert np.array_equal(scaled["out"]["f"][d], np.float32(2) * base["out"]["f"][d]), d
        assert np.array_equal(scaled["out"]["win_a"][d], base["out"]["win_a"][d]), d
        assert np.array_equal(scaled["out"]["win_x"][d], base["out"]["win_x"][d]), d


def test_landmark_coordinates_moved_off_their_points():
    # landmarks_in_x = 1 with coordinates that no longer equal X[l_xidx] (an
    # optimiser step on Lxyz, say): the per-sample bound is read from X, so
    # the values stay those of Def. 1 for the moved landmarks, which the
    # oracle computes by brute force without any bound
    X = synth.config_cloud(1)
    k = 4
    res = run_single(X, 64, k)
    rng = np.random.default_rng(31)
    moved = (res["Lxyz"] + rng.normal(0, 0.02, res["Lxyz"].shape)).astype(np.float32)
    Xd = torch.from_numpy(X).to(dev())
    pb = P.problem_from_complexes(Xd, [0, len(X)], torch.from_numpy(moved).to(dev()), [0, 64], [res["cx"]], k,
                                  l_xidx=torch.from_numpy(res["idx"].astype(np.int32)).to(dev()))
    run = P.filtration(pb)
    torch.cuda.synchronize()
    ref = OF.flood_all(X, moved, oracle_complex(res["cx"]), k, "brute")
    diam = OF.diameter(X)
    for d in range(4):
        got = run.f[d].cpu().numpy().astype(np.float64)
        assert np.abs(got - ref[d][0]).max() <= 1e-5 * diam, d
        wx = run.win_x[d].cpu().numpy()
        assert np.all((wx >= 0) & (wx < len(X))), d
    assert np.all(run.f[0].cpu().numpy() > 0)
