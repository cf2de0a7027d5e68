"""Pins of the oracle's mesh resolution and spin-image correlation
(oracle/matching.py) by closed forms, invariants and an independent library
query -- nothing here retypes the definitions."""
import math

import numpy as np
import pytest

from oracle import matching as Mt


def lattice(n, a, origin=(0.0, 0.0, 0.0)):
    g = np.arange(n) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return (np.stack([x, y, z], -1).reshape(-1, 3) + np.asarray(origin)).astype(np.float32)


def test_lattice_spacing_is_the_resolution():
    # every point of a cubic lattice of spacing a has its nearest other point at a
    X = lattice(6, 0.25, (3.0, -2.0, 7.5))
    d = Mt.nn_distances(X)
    assert np.all(d == 0.25)
    np.testing.assert_array_equal(Mt.nn_distances_tree(X), d)


def test_two_points_and_duplicates():
    X = np.array([[0, 0, 0], [3, 4, 0]], np.float32)
    np.testing.assert_array_equal(Mt.nn_distances(X), [5.0, 5.0])
    Y = np.array([[1, 1, 1], [1, 1, 1], [2, 1, 1]], np.float32)
    np.testing.assert_array_equal(Mt.nn_distances(Y), [0.0, 0.0, 1.0])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_equals_kdtree(seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (700, 3)).astype(np.float32)
    idx = rng.choice(700, 150, replace=False)
    np.testing.assert_allclose(Mt.nn_distances(X, idx), Mt.nn_distances_tree(X, idx),
                               rtol=1e-12)


def test_correlation_hand_example():
    # P = (1,2,3,4), Q = (1,3,2,6): N sum pq - sum p sum q = 4*37 - 10*12 = 28,
    # N sum p^2 - (sum p)^2 = 120 - 100 = 20, N sum q^2 - (sum q)^2 = 200 - 144 = 56,
    # R = 28 / sqrt(1120) = 7 / sqrt(70) = sqrt(70) / 10
    R = Mt.correlation([[1, 2, 3, 4]], [[1, 3, 2, 6]])
    assert abs(R[0, 0] - math.sqrt(70) / 10) < 1e-15


def test_correlation_invariants():
    rng = np.random.default_rng(4)
    A = rng.gamma(1.0, 2.0, (20, 64))
    B = rng.gamma(1.0, 2.0, (30, 64))
    R = Mt.correlation(A, B)
    assert np.all(np.abs(R) <= 1 + 1e-12)
    np.testing.assert_allclose(Mt.correlation(B, A), R.T, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.diag(Mt.correlation(A, A)), 1.0, rtol=1e-12)
    # R is unchanged by a positive affine map of either image; a negative one flips its sign
    np.testing.assert_allclose(Mt.correlation(3 * A + 7, B), R, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Mt.correlation(A, -0.5 * B + 1), -R, rtol=1e-10, atol=1e-12)
    # a constant image has no variance: R = 0 against everything
    assert np.all(Mt.correlation(np.full((1, 64), 2.0), B) == 0)


def test_best_match_recovers_a_permutation():
    rng = np.random.default_rng(5)
    A = rng.gamma(1.0, 2.0, (40, 256))
    perm = rng.permutation(40)
    j, r = Mt.best_match(A, A[perm])
    np.testing.assert_array_equal(perm[j], np.arange(40))
    np.testing.assert_allclose(r, 1.0, rtol=1e-12)


def test_normals_of_a_plane_and_a_sphere():
    rng = np.random.default_rng(8)
    # points on the plane z = 2: the normal is e_z, away from a viewpoint below
    P = np.c_[rng.uniform(0, 1, 400), rng.uniform(0, 1, 400), np.full(400, 2.0)].astype(np.float32)
    n, c, f, _ = Mt.estimate_normals(P, 0.2, (0.5, 0.5, -5.0))
    ok = ~f
    assert ok.sum() > 350
    np.testing.assert_allclose(n[ok], np.tile([0, 0, 1.0], (ok.sum(), 1)), atol=1e-9)
    # a unit sphere sampled densely: normals radial (outward from the centre)
    g = rng.normal(size=(3000, 3))
    S = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    n, c, f, _ = Mt.estimate_normals(S, 0.15, (0, 0, 0), idx=np.arange(300))
    cosang = (n * S[:300]).sum(1) / np.linalg.norm(S[:300], axis=1)
    assert np.all(cosang[~f] > 0.995)
    assert np.all(c >= 3)


def test_normals_counts_equal_brute_radius_counts():
    rng = np.random.default_rng(9)
    X = rng.uniform(0, 1, (500, 3)).astype(np.float32)
    _, c, _, _ = Mt.estimate_normals(X, 0.15, (0, 0, -1.0))
    from scipy.spatial import cKDTree
    t = cKDTree(X.astype(np.float64))
    ref = np.array([len(t.query_ball_point(p, 0.15 * (1 + 1e-12))) for p in X.astype(np.float64)])
    np.testing.assert_array_equal(c, ref)
