"""Seeded synthetic oriented-point scenes.

The paper's inputs are dense 3D objects given as oriented points, that is
positions with known surface normals (Section 2.1, the notation table; Table 2
lists the mesh-watermarking objects).  That data set is not available here, so
every scene is synthetic and drawn from a seeded ``numpy`` PCG64 generator:

* ``sphere_scene``: points on the unit sphere with Gaussian radial noise and
  analytic (radial) normals;
* ``primitives_scene``: random tori and ellipsoids with random radii, uniform
  random rotations, a per-object point density that varies tenfold, points
  sampled uniformly by area with analytic normals, each object's points in
  Morton order (mesh-file-like locality) and the objects concatenated in a
  random order;
* ``batch_specs`` / ``batch_scene``: many independent primitive scenes whose
  sizes are log-uniform.

All geometry is built in float64; normals are normalised in float64 and only
then rounded to float32, as are positions.  This module contains none of the
spin-image arithmetic; it is the one source of inputs shared by the HIP path's
tests and benchmarks and by the CPU oracle's tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng",
    "sphere_scene",
    "primitives_scene",
    "uniform_box_scene",
    "config_scene",
    "batch_specs",
    "batch_scene",
    "mean_nn_spacing",
    "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _finish(pts: np.ndarray, nrm: np.ndarray):
    nrm = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    return (np.ascontiguousarray(pts, dtype=np.float32),
            np.ascontiguousarray(nrm, dtype=np.float32))


def sphere_scene(M: int, seed: int = 1, noise_sigma: float = 0.005):
    """Unit sphere, x = (1 + e) u with u uniform on the sphere, e ~ N(0, sigma^2),
    normal n = u."""
    g = rng(seed)
    u = g.standard_normal((M, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    e = g.standard_normal(M) * noise_sigma if noise_sigma > 0 else np.zeros(M)
    pts = u * (1.0 + e)[:, None]
    return _finish(pts, u)


def uniform_box_scene(M: int, seed: int, box: float = 1.0):
    """Points uniform in [0, box]^3 with uniformly random unit normals (no
    surface structure; used for small randomized tests)."""
    g = rng(seed)
    pts = g.random((M, 3)) * box
    n = g.standard_normal((M, 3))
    return _finish(pts, n)


def _random_rotation(g: np.random.Generator) -> np.ndarray:
    q = g.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _ellipsoid_area(a, b, c):
    p = 1.6075  # Thomsen's approximation; used only to apportion point counts
    return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)


def _sample_ellipsoid(g, n, a, b, c):
    """Area-uniform points on the ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 by
    rejection from the unit sphere (acceptance = local area scale / its max)."""
    out_p, out_n, have = [], [], 0
    mn = min(a, b, c)
    while have < n:
        k = max(64, int((n - have) * 1.6) + 16)
        u = g.standard_normal((k, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        q = np.stack([u[:, 0] / a, u[:, 1] / b, u[:, 2] / c], axis=1)
        s = np.linalg.norm(q, axis=1) * mn
        keep = g.random(k) < s
        out_p.append(u[keep] * np.array([a, b, c]))
        out_n.append(q[keep])
        have += int(keep.sum())
    return np.concatenate(out_p)[:n], np.concatenate(out_n)[:n]


def _sample_torus(g, n, R, r):
    """Area-uniform points on a torus of major radius R, minor radius r."""
    out_p, out_n, have = [], [], 0
    while have < n:
        k = max(64, int((n - have) * 1.6) + 16)
        th = g.random(k) * 2 * math.pi
        ph = g.random(k) * 2 * math.pi
        keep = g.random(k) < (R + r * np.cos(th)) / (R + r)
        th, ph = th[keep], ph[keep]
        ring = R + r * np.cos(th)
        out_p.append(np.stack([ring * np.cos(ph), ring * np.sin(ph), r * np.sin(th)], axis=1))
        out_n.append(np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), np.sin(th)], axis=1))
        have += int(keep.sum())
    return np.concatenate(out_p)[:n], np.concatenate(out_n)[:n]


def _morton_order(p: np.ndarray) -> np.ndarray:
    lo = p.min(axis=0)
    span = np.maximum(p.max(axis=0) - lo, 1e-12)
    q = np.minimum((p - lo) / span * 1024.0, 1023).astype(np.uint64)
    code = np.zeros(len(p), dtype=np.uint64)
    for bit in range(10):
        for axis in range(3):
            code |= ((q[:, axis] >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + axis)
    return np.argsort(code, kind="stable")


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    share = weights / weights.sum() * total
    base = np.floor(share).astype(np.int64)
    short = total - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:short]] += 1
    return base


def primitives_scene(M: int, n_objects: int, seed: int, box: float = 10.0,
                     clusters: int = 0, cluster_sigma: float = 1.0,
                     radius_range=(0.2, 1.0), density_decades: float = 1.0):
    """Random tori and ellipsoids (probability 1/2 each).

    Ellipsoid semi-axes are each U(radius_range); a torus draws two values
    from U(radius_range) and uses the larger as major radius R and the smaller
    as minor radius r.  Each object gets a uniformly random rotation and a
    density 10^U(0, density_decades); its point count is proportional to
    density x area and the counts are rounded (largest remainder) to sum to M.
    Object centres are U(0, box)^3, or, with ``clusters`` = K > 0, K cluster
    centres U(box/8, 7 box/8)^3 and each object placed at a random cluster
    centre plus N(0, cluster_sigma^2 I), clipped to [0, box]^3.
    """
    g = rng(seed)
    lo_r, hi_r = radius_range
    objs = []
    if clusters > 0:
        cc = g.uniform(box / 8, 7 * box / 8, size=(clusters, 3))
    for _ in range(n_objects):
        kind = "torus" if g.random() < 0.5 else "ellipsoid"
        if kind == "ellipsoid":
            radii = g.uniform(lo_r, hi_r, size=3)
            area = _ellipsoid_area(*radii)
        else:
            two = g.uniform(lo_r, hi_r, size=2)
            radii = np.array([two.max(), two.min()])
            area = 4 * math.pi ** 2 * radii[0] * radii[1]
        rot = _random_rotation(g)
        if clusters > 0:
            c = cc[g.integers(clusters)] + g.standard_normal(3) * cluster_sigma
            centre = np.clip(c, 0.0, box)
        else:
            centre = g.uniform(0.0, box, size=3)
        dens = 10.0 ** g.uniform(0.0, density_decades)
        objs.append((kind, radii, rot, centre, dens * area))
    counts = _largest_remainder(np.array([o[4] for o in objs]), M)
    parts_p, parts_n = [], []
    for (kind, radii, rot, centre, _), n in zip(objs, counts):
        if n == 0:
            parts_p.append(np.zeros((0, 3)))
            parts_n.append(np.zeros((0, 3)))
            continue
        if kind == "ellipsoid":
            p, nn = _sample_ellipsoid(g, int(n), *radii)
        else:
            p, nn = _sample_torus(g, int(n), *radii)
        p = p @ rot.T + centre
        nn = nn @ rot.T
        o = _morton_order(p)
        parts_p.append(p[o])
        parts_n.append(nn[o])
    order = g.permutation(n_objects)
    pts = np.concatenate([parts_p[i] for i in order])
    nrm = np.concatenate([parts_n[i] for i in order])
    return _finish(pts, nrm)


@dataclass(frozen=True)
class SceneConfig:
    name: str
    M: int
    N: int            # oriented points are indices 0..N-1 (the first N points)
    W: int
    bin: float
    support_angle: float
    seed: int


# Spin-image parameters are W (pixels per side), bin size (scene units) and
# support angle (radians); the 60-degree angle is stored as float32(pi/3).
CONFIGS = {
    "sphere2k": SceneConfig("sphere2k", 2000, 2000, 16, 0.05, float(np.float32(math.pi / 3)), 1),
    "prims100k": SceneConfig("prims100k", 100_000, 65_536, 32, 0.02, float(np.float32(math.pi / 3)), 2),
    "clustered2m": SceneConfig("clustered2m", 2_000_000, 2_000_000, 32, 0.02, float(np.float32(math.pi / 3)), 3),
    # the shape of the paper's experiments (826K points, the first 10 % oriented,
    # W = 5, B = 0.1 x mesh resolution, S = 2 pi, brute force): bin is NaN here
    # and is 0.1 x mean_nn_spacing of the generated points
    "paper826k": SceneConfig("paper826k", 826_000, 82_600, 5, float("nan"),
                             float(np.float32(2 * math.pi)), 10),
}


def config_scene(name: str, M: int | None = None):
    """Scene of a named workload; ``M`` overrides the point count (smaller
    stand-ins for tests keep the recipe but not the size)."""
    cfg = CONFIGS[name]
    m = cfg.M if M is None else int(M)
    if name == "sphere2k":
        return sphere_scene(m, cfg.seed)
    if name == "prims100k":
        return primitives_scene(m, 20, cfg.seed, box=10.0)
    if name == "clustered2m":
        return primitives_scene(m, 400, cfg.seed, box=40.0, clusters=16, cluster_sigma=1.0)
    if name == "paper826k":
        return primitives_scene(m, 165, cfg.seed, box=20.0)
    raise KeyError(name)


def mean_nn_spacing(xyz: np.ndarray, sample: int = 20_000, seed: int = 0) -> float:
    """Mean distance from a point to its nearest other point (the "mesh
    resolution"), estimated on a seeded sample of the points."""
    from scipy.spatial import cKDTree
    pts = np.asarray(xyz, dtype=np.float64)
    tree = cKDTree(pts)
    idx = rng(seed).choice(len(pts), min(sample, len(pts)), replace=False)
    d, _ = tree.query(pts[idx], k=2)
    return float(d[:, 1].mean())


def batch_specs(n_scenes: int = 256, base_seed: int = 4000,
                m_range=(1_000, 200_000), widths=(16, 32, 64)):
    """(seed, M_s, W_s) per scene: M_s = round(exp(U(ln lo, ln hi))) and W_s
    uniform over ``widths``, each drawn from the scene's own generator."""
    out = []
    for s in range(n_scenes):
        g = rng(base_seed + s)
        m = int(round(math.exp(g.uniform(math.log(m_range[0]), math.log(m_range[1])))))
        w = int(widths[g.integers(len(widths))])
        out.append((base_seed + s, m, w))
    return out


def batch_scene(seed: int, M: int):
    """One scene of the batch: the 20-primitive [0, 10]^3 generator."""
    return primitives_scene(M, 20, seed, box=10.0)
