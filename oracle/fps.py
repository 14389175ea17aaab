"""Farthest-point landmark selection (oracle; test infrastructure).

Greedy k-centre (Sec. 3.2, "Theoretical results": FPS is a 2-approximation
of the optimal covering radius).  The arithmetic recipe is fixed in
float32 so that a GPU implementation can match the indices bit for bit:
dx = x - l rounded to float32 per axis; d2 = (dx*dx + dy*dy) + dz*dz with
every product and sum rounded to float32 and no fused multiply-add;
mind_i = min(mind_i, d2); next landmark = argmax mind, lowest index on
ties; start index given (0 in every workload here).
"""
import numpy as np

from . import native


class FPSDegenerate(ValueError):
    pass


def fps(X: np.ndarray, n_landmarks: int, start: int = 0, nthreads=None):
    """Returns (idx int32 [L], radius float32 [L]) where radius[t] is the
    covering radius max_i min_{s<=t} ||x_i - l_s|| after t+1 landmarks
    (float32 sqrt of the recipe's squared distance)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    idx = np.zeros(n_landmarks, np.int32)
    rad = np.zeros(n_landmarks, np.float32)
    rc = native.lib().or_fps(native.ptr(X), X.shape[0], int(start), int(n_landmarks),
                             native.ptr(idx), native.ptr(rad), native.threads(nthreads))
    if rc == 4:
        raise FPSDegenerate("fewer distinct points than landmarks")
    if rc != 0:
        raise ValueError("or_fps failed: %d" % rc)
    return idx, rad


def fps_python(X: np.ndarray, n_landmarks: int, start: int = 0):
    """Pure numpy float32 version of the same recipe (numpy float32 ops are
    correctly rounded and never fused).  Slow; small inputs only."""
    X = np.asarray(X, dtype=np.float32)
    def d2(l):
        d = X - l
        s = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
        return s + d[:, 2] * d[:, 2]
    idx = [start]
    mind = d2(X[start])
    rad = []
    for t in range(1, n_landmarks + 1):
        m = mind.max()
        rad.append(np.sqrt(m))
        if t == n_landmarks:
            break
        nxt = int(np.flatnonzero(mind == m)[0])
        idx.append(nxt)
        mind = np.minimum(mind, d2(X[nxt]))
    return np.array(idx, np.int32), np.array(rad, np.float32)


def fps_fp64(X: np.ndarray, n_landmarks: int, start: int = 0):
    """Same greedy rule in float64 -- information only (reports where the
    float32 recipe and exact-ish arithmetic first choose differently)."""
    X = np.asarray(X, dtype=np.float64)
    idx = [start]
    mind = ((X - X[start]) ** 2).sum(1)
    for _ in range(1, n_landmarks):
        nxt = int(np.argmax(mind))
        idx.append(nxt)
        mind = np.minimum(mind, ((X - X[nxt]) ** 2).sum(1))
    return np.array(idx, np.int32)
