"""Plain FP64 definitions of the workloads next to spin-image generation.

TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP library.

* Mesh resolution.  The paper sets the bin size B as a factor of the mesh
  resolution (Section 2.1, the notation table), which it does not define
  further; the reading here is the usual one for point sets: the mean, over
  the chosen points, of the distance from a point to its nearest other point
  of the scene.  ``nn_distances`` is that distance by brute force;
  ``nn_distances_tree`` the same through SciPy's k-d tree (a library
  nearest-neighbour query), for scenes too large to brute-force.
* Spin-image matching.  The paper cites the use of spin images for object
  recognition (Johnson and Hebert), where images are compared by the
  normalised linear correlation coefficient of their bins; here over all
  N = W x W bins:
      R(P, Q) = (N sum p q - sum p sum q)
                / sqrt((N sum p^2 - (sum p)^2) (N sum q^2 - (sum q)^2)).
  Reading: an image whose bins are all equal (zero variance, e.g. empty) has
  R = 0 with every image.  ``best_match`` takes, for each image of A, the
  image of B of largest R (the lowest index on ties).
"""
from __future__ import annotations

import numpy as np


def nn_distances(xyz, idx=None, block: int = 256) -> np.ndarray:
    """Distance from each chosen point to its nearest other point, FP64 brute
    force (points are FP32, widened exactly).  Another point at the same
    place gives 0."""
    X = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    idx = np.arange(len(X)) if idx is None else np.asarray(idx, dtype=np.int64)
    out = np.empty(len(idx))
    for a in range(0, len(idx), block):
        q = idx[a:a + block]
        d2 = ((X[None, :, :] - X[q][:, None, :]) ** 2).sum(axis=2)
        d2[np.arange(len(q)), q] = np.inf   # not the point itself
        out[a:a + block] = np.sqrt(d2.min(axis=1))
    return out


def nn_distances_tree(xyz, idx=None) -> np.ndarray:
    from scipy.spatial import cKDTree
    X = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    idx = np.arange(len(X)) if idx is None else np.asarray(idx, dtype=np.int64)
    tree = cKDTree(X)
    d, j = tree.query(X[idx], k=2)
    # k = 2: the first neighbour is the point itself (or a duplicate at 0)
    return np.where(j[:, 0] == idx, d[:, 1], d[:, 0])


def correlation(A, B) -> np.ndarray:
    """R for every pair (rows of A against rows of B), FP64."""
    A = np.asarray(A, dtype=np.float64).reshape(len(A), -1)
    B = np.asarray(B, dtype=np.float64).reshape(len(B), -1)
    N = A.shape[1]
    sa, sb = A.sum(1), B.sum(1)
    va = N * (A * A).sum(1) - sa * sa
    vb = N * (B * B).sum(1) - sb * sb
    num = N * (A @ B.T) - np.outer(sa, sb)
    den = np.sqrt(np.outer(np.maximum(va, 0.0), np.maximum(vb, 0.0)))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def best_match(A, B):
    """(index of the best image of B for each row of A, its R)."""
    R = correlation(A, B)
    j = np.argmax(R, axis=1)
    return j, R[np.arange(len(R)), j]


# ---------------------------------------------------------------------------
# Normal estimation.  The paper takes oriented points with known normals
# (Section 2.1); for raw points the usual estimate is the direction of least
# spread of the neighbourhood.  Reading: the neighbours of p are the points x
# with |x - p| <= r, p itself included; their covariance (about their
# centroid, divided by their count) has eigenvalues l0 <= l1 <= l2, and the
# normal is the unit eigenvector of l0, signed so that n . (p - v) >= 0 for a
# given viewpoint v (pointing away from v).  A neighbour within band
# (relative) of the sphere, |x - p|^2 / r^2 - 1| < band, could be counted
# either way at FP32 distance precision: such points are flagged, as are
# points whose two smallest eigenvalues are too close for the direction to be
# defined ((l1 - l0) / max(l2, tiny) < gap) and points with
# |n . (p - v)| < 1e-6 |p - v| (sign undefined).
# ---------------------------------------------------------------------------
def estimate_normals(xyz, radius: float, viewpoint, idx=None, band: float = 1e-5,
                     gap: float = 1e-4, block: int = 128):
    """(normals (n, 3), neighbour counts (n,), flagged (n,) bool, eigenvalue
    gap (l1 - l0) / l2 (n,)) for the chosen points, FP64, brute-force
    neighbourhoods.  The gap bounds how far rounding of the inputs can turn
    the normal: about (relative error of the covariance) / gap radians."""
    X = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    idx = np.arange(len(X)) if idx is None else np.asarray(idx, dtype=np.int64)
    r2 = float(np.float32(radius)) ** 2
    v = np.asarray(viewpoint, dtype=np.float32).astype(np.float64)
    normals = np.zeros((len(idx), 3))
    counts = np.zeros(len(idx), dtype=np.int64)
    flag = np.zeros(len(idx), dtype=bool)
    gaps = np.zeros(len(idx))
    for a in range(0, len(idx), block):
        q = idx[a:a + block]
        d2 = ((X[None, :, :] - X[q][:, None, :]) ** 2).sum(axis=2)
        for t, i in enumerate(q):
            near = d2[t] <= r2
            flag[a + t] |= bool((np.abs(d2[t] / r2 - 1.0) < band).any())
            nb = X[near]
            counts[a + t] = len(nb)
            c = nb.mean(axis=0)
            C = (nb - c).T @ (nb - c) / len(nb)
            lam, vec = np.linalg.eigh(C)
            n = vec[:, 0]
            gaps[a + t] = (lam[1] - lam[0]) / max(lam[2], 1e-300)
            if gaps[a + t] < gap:
                flag[a + t] = True
            s = float(n @ (X[i] - v))
            if abs(s) < 1e-6 * np.linalg.norm(X[i] - v):
                flag[a + t] = True
            normals[a + t] = n if s >= 0 else -n
    return normals, counts, flag, gaps
