"""Surface samplers and the five workload recipes (see package docstring)."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------------------
# primitive surfaces, uniform in area


def sphere_surface(rng: np.random.Generator, n: int, center, radius: float) -> np.ndarray:
    """n points uniform on a sphere: normalised Gaussian directions."""
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.asarray(center, dtype=np.float64) + radius * d


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([
        math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
        math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
        math.sqrt(u1) * math.sin(2 * math.pi * u3),
        math.sqrt(u1) * math.cos(2 * math.pi * u3),
    ])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def torus_surface(rng: np.random.Generator, n: int, center, R: float, r: float,
                  rot: np.ndarray | None = None) -> np.ndarray:
    """n points uniform in area on a torus (major R, minor r).

    The area element is r (R + r cos v) du dv, so (u, v) uniform is
    thinned by acceptance (R + r cos v) / (R + r).
    """
    out = np.empty((0, 2))
    while out.shape[0] < n:
        m = int((n - out.shape[0]) * (R + r) / R * 1.1) + 16
        u = rng.random(m) * 2 * math.pi
        v = rng.random(m) * 2 * math.pi
        keep = rng.random(m) < (R + r * np.cos(v)) / (R + r)
        out = np.concatenate([out, np.stack([u[keep], v[keep]], 1)])
    u, v = out[:n, 0], out[:n, 1]
    p = np.stack([(R + r * np.cos(v)) * np.cos(u),
                  (R + r * np.cos(v)) * np.sin(u),
                  r * np.sin(v)], 1)
    if rot is not None:
        p = p @ rot.T
    return np.asarray(center, dtype=np.float64) + p


def box_surface(rng: np.random.Generator, n: int, center, sides) -> np.ndarray:
    """n points uniform on the surface of an axis-aligned box."""
    a = np.asarray(sides, dtype=np.float64)
    areas = np.array([a[1] * a[2], a[1] * a[2], a[0] * a[2], a[0] * a[2],
                      a[0] * a[1], a[0] * a[1]])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    p = (rng.random((n, 3)) - 0.5) * a
    axis = face // 2
    sign = np.where(face % 2 == 0, -0.5, 0.5)
    p[np.arange(n), axis] = sign * a[axis]
    return np.asarray(center, dtype=np.float64) + p


# ----------------------------------------------------------------------------
# primitive mixes in the unit cube


@dataclass
class Primitive:
    kind: str
    center: np.ndarray
    params: tuple
    rot: np.ndarray | None
    area: float


def _draw_primitive(rng: np.random.Generator, kind: str) -> Primitive:
    if kind == "sphere":
        r = rng.uniform(0.05, 0.2)
        c = rng.uniform(r, 1 - r, 3)
        return Primitive(kind, c, (r,), None, 4 * math.pi * r * r)
    if kind == "torus":
        R = rng.uniform(0.1, 0.25)
        r = R * rng.uniform(0.2, 0.4)
        c = rng.uniform(R + r, 1 - R - r, 3)
        return Primitive(kind, c, (R, r), random_rotation(rng), 4 * math.pi ** 2 * R * r)
    if kind == "box":
        s = rng.uniform(0.1, 0.4, 3)
        c = rng.uniform(s / 2, 1 - s / 2)
        return Primitive(kind, c, tuple(s), None,
                         2 * (s[0] * s[1] + s[1] * s[2] + s[0] * s[2]))
    raise ValueError(kind)


def _sample(rng: np.random.Generator, p: Primitive, n: int) -> np.ndarray:
    if p.kind == "sphere":
        return sphere_surface(rng, n, p.center, p.params[0])
    if p.kind == "torus":
        return torus_surface(rng, n, p.center, p.params[0], p.params[1], p.rot)
    return box_surface(rng, n, p.center, p.params)


def primitive_mix(rng: np.random.Generator, n: int, kinds, noise: float) -> np.ndarray:
    """Union of primitives in [0,1]^3; points split in proportion to area
    (uniform surface density); Gaussian noise added after sampling."""
    prims = [_draw_primitive(rng, k) for k in kinds]
    areas = np.array([p.area for p in prims])
    counts = np.floor(n * areas / areas.sum()).astype(np.int64)
    counts[np.argmax(areas)] += n - counts.sum()
    pts = np.concatenate([_sample(rng, p, int(c)) for p, c in zip(prims, counts)])
    pts += rng.normal(0.0, noise, pts.shape)
    pts = pts[rng.permutation(n)]
    return np.ascontiguousarray(pts, dtype=np.float32)


# ----------------------------------------------------------------------------
# the five workloads


@dataclass(frozen=True)
class CloudConfig:
    name: str
    n_points: int
    n_landmarks: int
    k: int
    seed: int


CONFIGS = {
    1: CloudConfig("torus_N2k_L64_k4", 2_000, 64, 4, 1001),
    2: CloudConfig("mix5_N1M_L2000_k10", 1_000_000, 2_000, 10, 1002),
    3: CloudConfig("mix20_N10M_L10000_k8", 10_000_000, 10_000, 8, 1003),
    4: CloudConfig("batch512_logU10k-500k_L1pct_k6", 0, 0, 6, 1004),
    5: CloudConfig("twotorus64_N100k_L512_k6", 100_000, 512, 6, 1005),
}


def config_cloud(cfg: int, n_points: int | None = None) -> np.ndarray:
    """The single-cloud workloads 1-3 (optionally at another size with the
    same recipe, for tests)."""
    c = CONFIGS[cfg]
    n = c.n_points if n_points is None else int(n_points)
    rng = np.random.Generator(np.random.PCG64(c.seed))
    if cfg == 1:
        p = torus_surface(rng, n, (0.0, 0.0, 0.0), 1.0, 0.3)
        p += rng.normal(0.0, 0.01, p.shape)
        return np.ascontiguousarray(p, dtype=np.float32)
    if cfg == 2:
        return primitive_mix(rng, n, ["sphere"] * 2 + ["torus"] * 2 + ["box"], 0.002)
    if cfg == 3:
        return primitive_mix(rng, n, ["sphere"] * 8 + ["torus"] * 8 + ["box"] * 4, 0.001)
    raise ValueError("configs 4 and 5 are multi-cloud: use batched_clouds / differentiable_clouds")


def batched_clouds(n_clouds: int = 512, seed: int = 1004, n_min: int = 10_000,
                   n_max: int = 500_000, scale: float = 1.0):
    """Workload 4: clouds with N log-uniform in [n_min, n_max], each a union
    of 1-6 primitives of uniform random type, noise 0.002; L = min(1% of N,
    4096).  Returns (list of [N_i,3] float32 arrays, list of L_i).
    `scale` shrinks every N_i (tests use it to keep sizes small)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    clouds, lms = [], []
    for _ in range(n_clouds):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n = max(16, int(round(n * scale)))
        m = int(rng.integers(1, 7))
        kinds = list(rng.choice(["sphere", "torus", "box"], size=m))
        clouds.append(primitive_mix(rng, n, kinds, 0.002))
        lms.append(max(8, min(n // 100, 4096)))
    return clouds, lms


def differentiable_clouds(n_clouds: int = 64, n_points: int = 100_000, seed: int = 1005):
    """Workload 5: unions of two randomly placed and oriented tori, noise 0.005."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [primitive_mix(rng, n_points, ["torus", "torus"], 0.005) for _ in range(n_clouds)]


def circle_points(n: int) -> np.ndarray:
    """n equally spaced points on the unit circle in the plane z=0 (float32)."""
    t = 2 * np.pi * np.arange(n) / n
    return np.ascontiguousarray(np.stack([np.cos(t), np.sin(t), np.zeros(n)], 1), dtype=np.float32)


def lattice_points(side: int, seed: int = 7) -> np.ndarray:
    """The integer lattice {0..side-1}^3 in a seeded random row order: every
    distance is a small integer norm, so exact ties are everywhere."""
    g = np.arange(side, dtype=np.float32)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    return np.ascontiguousarray(X[np.random.default_rng(seed).permutation(len(X))])


def swisscheese(n_points: int = 1_000_000, n_voids: int = 10, seed: int = 2000, side: float = 5.0):
    """A swiss-cheese cloud as the paper's synthetic classification dataset
    is described (Sec. 5.3): points uniform in [0, side]^3 minus n_voids
    disjoint balls with radii uniform in [0.1, 0.5] and uniform centres (each
    ball inside the cube; a ball overlapping an earlier one is redrawn).
    Returns (float32 [n_points, 3], centres [n_voids, 3], radii [n_voids])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cs, rs = [], []
    while len(cs) < n_voids:
        r = rng.uniform(0.1, 0.5)
        c = rng.uniform(r, side - r, 3)
        if all(np.linalg.norm(c - c2) > r + r2 for c2, r2 in zip(cs, rs)):
            cs.append(c)
            rs.append(r)
    C = np.array(cs).reshape(-1, 3)
    R = np.array(rs)
    out = []
    have = 0
    while have < n_points:
        m = int((n_points - have) * 1.05) + 64
        p = rng.random((m, 3)) * side
        keep = np.ones(m, dtype=bool)
        for c, r in zip(C, R):
            keep &= ((p - c) ** 2).sum(1) > r * r
        p = p[keep]
        out.append(p)
        have += len(p)
    X = np.concatenate(out)[:n_points]
    return np.ascontiguousarray(X, dtype=np.float32), C, R


def planar_cheese(n_points: int = 100_000, n_voids: int = 10, seed: int = 2100, side: float = 5.0):
    """The swiss-cheese recipe in the plane (ambient dimension 2): points
    uniform in [0, side]^2 minus n_voids disjoint disks with radii uniform in
    [0.1, 0.5].  Returns float32 [n_points, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cs, rs = [], []
    while len(cs) < n_voids:
        r = rng.uniform(0.1, 0.5)
        c = rng.uniform(r, side - r, 2)
        if all(np.linalg.norm(c - c2) > r + r2 for c2, r2 in zip(cs, rs)):
            cs.append(c)
            rs.append(r)
    out, have = [], 0
    while have < n_points:
        m = int((n_points - have) * 1.1) + 64
        p = rng.random((m, 2)) * side
        keep = np.ones(m, dtype=bool)
        for c, r in zip(cs, rs):
            keep &= ((p - c) ** 2).sum(1) > r * r
        out.append(p[keep])
        have += int(keep.sum())
    return np.ascontiguousarray(np.concatenate(out)[:n_points], dtype=np.float32)
