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


def test_3d_matches_scipy_kdtree_with_coincident_points(ora):
    """Sec. 3.1 prefers neighbours counted in 3D: the distance in space."""
    from scipy.spatial import cKDTree

    g = synth.rng(75)
    x, y, z = g.uniform(-1, 1, 2000), g.uniform(-1, 1, 2000), g.uniform(-1, 1, 2000)
    x[50:56], y[50:56], z[50:56] = x[3], y[3], z[3]  # seven coincident particles
    x[60], y[60] = x[4], y[4]  # same projection as particle 4, apart in z
    pts = np.column_stack([x, y, z])
    d, _ = cKDTree(pts).query(pts, k=33)
    for k in (1, 6, 7, 32):
        np.testing.assert_allclose(ora.knn(x, y, k, z=z), d[:, k], rtol=1e-15, atol=0)
    assert ora.knn(x, y, 1)[4] == 0.0 and ora.knn(x, y, 1, z=z)[4] > 0.0
    # z = 0 everywhere is the 2D definition, to the bit
    np.testing.assert_array_equal(ora.knn(x, y, 8, z=np.zeros_like(z)), ora.knn(x, y, 8))


def shell_distance_3d(k, reach=5):
    a = np.arange(-reach, reach + 1)
    A, B, C = np.meshgrid(a, a, a)
    r2 = (A * A + B * B + C * C).ravel()
    return np.sqrt(np.sort(r2[r2 > 0])[k - 1])


def test_3d_integer_lattice_shells(ora):
    n = 11
    ix, iy, iz = (v.ravel() for v in np.meshgrid(np.arange(n), np.arange(n), np.arange(n)))
    x, y, z = ix.astype(float), iy.astype(float), iz.astype(float)
    interior = np.all([(v >= 3) & (v <= n - 4) for v in (ix, iy, iz)], axis=0)
    # shells of the cubic lattice: 6 at 1, 12 at sqrt 2, 8 at sqrt 3, 6 at 2, 24 at sqrt 5
    for k in (1, 6, 7, 18, 19, 26, 27, 32, 33, 56):
        s = ora.knn(x, y, k, z=z)
        assert np.all(s[interior] == shell_distance_3d(k)), k
    assert shell_distance_3d(26) == np.sqrt(3.0) and shell_distance_3d(27) == 2.0


@pytest.mark.parametrize("dim", [2, 3])
def test_species_are_smoothed_separately(ora, dim):
    """Sec. 3.1: with several species, a particle's smoothing length counts
    only neighbours of its own species."""
    from scipy.spatial import cKDTree

    g = synth.rng(77 + dim)
    n = 3000
    x, y, z = g.normal(size=n), g.normal(size=n), g.normal(size=n)
    sp = np.where(g.random(n) < 0.1, 7, np.where(g.random(n) < 0.5, 0, 2)).astype(np.int32)
    zz = z if dim == 3 else None
    s = ora.knn(x, y, 16, z=zz, species=sp)
    for lab in (0, 2, 7):
        m = sp == lab
        pts = np.column_stack([x[m], y[m]] + ([z[m]] if dim == 3 else []))
        d, _ = cKDTree(pts).query(pts, k=17)
        np.testing.assert_allclose(s[m], d[:, 16], rtol=1e-15, atol=0)
    # the same labels in another numbering give the same lengths
    np.testing.assert_array_equal(ora.knn(x, y, 16, z=zz, species=(sp + 3) * 5), s)
    # a species with no more than k particles has no k-th neighbour
    sp2 = sp.copy()
    sp2[:16] = 99
    with pytest.raises(ValueError):
        ora.knn(x, y, 16, z=zz, species=sp2)
