"""Pins for the oracle's farthest-point sampling (greedy k-centre)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import fps as F


def test_c_matches_numpy_recipe():
    X = synth.config_cloud(1)
    a = F.fps(X, 64)
    b = F.fps_python(X, 64)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("j,stages", [(8, 6), (10, 7)])
def test_circle_dyadic_stages(j, stages):
    # Appendix circle example: from angle 0, stage s adds the points at odd
    # multiples of 2 pi / 2^s; after 2^s picks the set is {multiples of N/2^s}.
    N = 2 ** j
    X = synth.circle_points(N)
    idx, rad = F.fps(X, 2 ** stages)
    for s in range(1, stages + 1):
        got = set(idx[: 2 ** s].tolist())
        assert got == set(range(0, N, N // 2 ** s)), s
    # covering radius after 2^s picks is the chord to the half-arc midpoint
    for s in range(1, stages):
        chord = 2 * np.sin(np.pi / 2 ** (s + 1))
        assert abs(rad[2 ** s - 1] - chord) < 1e-5


def _kcenter_opt(X, k):
    best = np.inf
    D = np.sqrt(((X[:, None] - X[None]) ** 2).sum(-1))
    for S in itertools.combinations(range(len(X)), k):
        best = min(best, D[:, S].min(1).max())
    return best


@pytest.mark.parametrize("seed", range(12))
def test_two_approximation(seed):
    # greedy k-centre covers within twice the optimum (Sec. 2)
    rng = np.random.default_rng(seed)
    X = rng.random((11, 3)).astype(np.float32)
    for k in (1, 2, 3):
        idx, rad = F.fps(X, k)
        opt = _kcenter_opt(X.astype(np.float64), k)
        assert rad[-1] <= 2 * opt * (1 + 1e-6)
        assert len(set(idx.tolist())) == k


def test_radius_sequence():
    X = synth.config_cloud(1)
    idx, rad = F.fps(X, 64)
    assert np.all(np.diff(rad) <= 0)
    X64 = X.astype(np.float64)
    for t in (0, 5, 31, 63):
        d = np.sqrt(((X64[:, None] - X64[idx[: t + 1]][None]) ** 2).sum(-1)).min(1)
        assert abs(d.max() - rad[t]) <= 1e-6 * (1 + d.max())
        # landmark t+1 is the farthest point from the first t+1
        if t + 1 < 64:
            assert abs(d[idx[t + 1]] - d.max()) <= 1e-6


def test_degenerate_duplicates():
    X = np.repeat(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), 5, axis=0)
    F.fps(X, 3)
    with pytest.raises(F.FPSDegenerate):
        F.fps(X, 4)


def test_fp64_variant_agrees_where_float32_is_exact():
    # integer coordinates below 2^7: every difference, square and sum of the
    # float32 recipe is exact, so the FP64 greedy rule must pick the same
    # landmarks (ties included: both take the lowest index)
    X = synth.lattice_points(12).astype(np.float32)
    a, _ = F.fps(X, 200)
    b = F.fps_fp64(X, 200)
    assert np.array_equal(a, b)
    rng = np.random.default_rng(4)
    Y = rng.integers(0, 100, (3000, 3)).astype(np.float32)
    assert np.array_equal(F.fps(Y, 300)[0], F.fps_fp64(Y, 300))


def test_fp64_variant_on_the_torus():
    # off the lattice the two may part ways late; they agree on the start
    # and (for this cloud) on the first landmarks
    X = synth.config_cloud(1)
    a, _ = F.fps(X, 64)
    b = F.fps_fp64(X, 64)
    first = int(np.argmax(a != b)) if np.any(a != b) else 64
    assert first >= 8
