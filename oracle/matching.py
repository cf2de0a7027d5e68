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
