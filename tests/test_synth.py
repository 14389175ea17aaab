"""The seeded input generators: shapes and invariants of the recipes."""
import numpy as np

import synth


def test_swisscheese_recipe():
    X, C, R = synth.swisscheese(50_000, 12, seed=3)
    assert X.shape == (50_000, 3) and X.dtype == np.float32
    assert X.min() >= 0.0 and X.max() <= 5.0
    assert len(C) == 12 and np.all((R >= 0.1) & (R <= 0.5))
    # balls inside the cube and pairwise disjoint
    assert np.all(C - R[:, None] >= 0) and np.all(C + R[:, None] <= 5.0)
    for i in range(12):
        for j in range(i):
            assert np.linalg.norm(C[i] - C[j]) > R[i] + R[j]
    # no point inside a void
    X64 = X.astype(np.float64)
    for c, r in zip(C, R):
        assert np.all(((X64 - c) ** 2).sum(1) > r * r * (1 - 1e-6))
    # deterministic by seed
    X2, _, _ = synth.swisscheese(50_000, 12, seed=3)
    assert np.array_equal(X, X2)
    assert not np.array_equal(X, synth.swisscheese(50_000, 12, seed=4)[0])
