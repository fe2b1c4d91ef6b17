"""Pins of the smoothing-length oracle (Sec. 3.1: the smoothing length of a
particle is the radius holding its N_sph nearest neighbours; in 2D, the
distance to the k-th nearest other particle)."""
import numpy as np
import pytest

import synth


def test_matches_scipy_kdtree_with_coincident_points(ora):
    from scipy.spatial import cKDTree

    g = synth.rng(71)
    x, y = g.uniform(-1, 1, 2500), g.uniform(-1, 1, 2500)
    x[100:110], y[100:110] = x[5], y[5]  # eleven coincident particles
    pts = np.column_stack([x, y])
    d, _ = cKDTree(pts).query(pts, k=33)
    for k in (1, 8, 32):
        # scipy lists the particle itself (distance 0) first
        np.testing.assert_allclose(ora.knn(x, y, k), d[:, k], rtol=1e-15, atol=0)
    # among eleven coincident particles the ten nearest others are at distance 0
    s = ora.knn(x, y, 10)
    assert np.all(s[[5] + list(range(100, 110))] == 0.0)
    assert ora.knn(x, y, 11)[5] > 0.0


def shell_distance(k, reach=8):
    """k-th smallest |v| over nonzero integer vectors v (lattice shells)."""
    a = np.arange(-reach, reach + 1)
    A, B = np.meshgrid(a, a)
    r2 = (A * A + B * B).ravel()
    return np.sqrt(np.sort(r2[r2 > 0])[k - 1])


def test_integer_lattice_shells(ora):
    n = 25
    ix, iy = np.meshgrid(np.arange(n), np.arange(n))
    x, y = ix.ravel().astype(float), iy.ravel().astype(float)
    interior = (ix.ravel() >= 6) & (ix.ravel() <= n - 7) & (iy.ravel() >= 6) & (iy.ravel() <= n - 7)
    for k in (1, 4, 5, 8, 9, 12, 13, 20, 21, 24, 25, 28, 29, 32):
        s = ora.knn(x, y, k)
        assert np.all(s[interior] == shell_distance(k)), k
    # a corner point: neighbours only in one quadrant
    s = ora.knn(x, y, 3)
    assert s[0] == np.sqrt(2.0)  # (1,0), (0,1), then (1,1)


def test_two_particles_and_bad_k(ora):
    s = ora.knn(np.array([0.0, 3.0]), np.array([0.0, 4.0]), 1)
    assert np.all(s == 5.0)
    with pytest.raises(ValueError):
        ora.knn(np.array([0.0, 1.0]), np.array([0.0, 0.0]), 2)


def test_query_subset_matches_full(ora):
    g = synth.rng(73)
    x, y = g.normal(size=1500), g.normal(size=1500)
    at = np.array([0, 7, 1499, 7, 300])
    np.testing.assert_array_equal(ora.knn(x, y, 16, at=at), ora.knn(x, y, 16)[at])
