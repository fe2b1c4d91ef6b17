"""GPU smoothing lengths (Sec. 3.1: distance to the k-th nearest other
particle) against the brute-force oracle.  Both form every squared distance
in FP64 exactly as written, so the k-th distance agrees to the last bit
(the square root of the same FP64 value; 1 ulp is allowed for the device
square root)."""
import numpy as np
import pytest

import synth
from gpu_helpers import dev, say

pytestmark = pytest.mark.gpu


def gpu_knn(x, y, k, leaf=16):
    import paper_1312_1128_amd as g
    import torch

    s = g.smoothing_lengths(dev(x), dev(y), k=k, leaf_size=leaf)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def clustered(n, seed):
    """Uniform points, a dense clump, exact duplicates, and a sparse halo."""
    g = synth.rng(seed)
    x = np.concatenate([g.uniform(-1, 1, n // 2), g.normal(0.3, 1e-3, n // 4), g.normal(0, 5, n - n // 2 - n // 4)])
    y = np.concatenate([g.uniform(-1, 1, n // 2), g.normal(-0.2, 1e-3, n // 4), g.normal(0, 5, n - n // 2 - n // 4)])
    x[10:30], y[10:30] = x[3], y[3]  # 21 coincident particles
    return x, y


@pytest.mark.parametrize("k,leaf", [(1, 16), (8, 4), (16, 16), (32, 16), (33, 8), (64, 64)])
def test_knn_matches_oracle(ora, k, leaf):
    x, y = clustered(9001, 81)  # ragged last group of 41
    say(f"[gpu] knn n={x.size} k={k} leaf={leaf}")
    got = gpu_knn(x, y, k, leaf)
    ref = ora.knn(x, y, k)
    np.testing.assert_array_max_ulp(got, ref, maxulp=1)
    if k <= 20:
        assert np.all(got[[3] + list(range(10, 30))] == 0.0)


def test_knn_nfw_halo_sampled(ora):
    """The 1e6-particle NFW halo of the headline workload: 2048 sampled
    particles against the brute force, and all of them against the host
    k-d tree the inputs are made with."""
    lens = synth.nfw_halo(1_000_000, synth.BASE_SEED + 2)
    say(f"[gpu] knn nfw n={lens.n}")
    got = gpu_knn(lens.x, lens.y, 32)
    at = synth.sample_rays(lens.x, lens.y, 2048, 83)
    np.testing.assert_array_max_ulp(got[at], ora.knn(lens.x, lens.y, 32, at=at), maxulp=1)
    np.testing.assert_allclose(got, lens.s, rtol=1e-15, atol=0)


def test_knn_small_and_invalid():
    import paper_1312_1128_amd as g

    np.testing.assert_array_equal(gpu_knn(np.array([0.0, 3.0]), np.array([0.0, 4.0]), 1), [5.0, 5.0])
    g0 = synth.rng(85)
    x, y = g0.uniform(size=65), g0.uniform(size=65)
    s = gpu_knn(x, y, 64)  # every other particle counts: the farthest one
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    np.testing.assert_allclose(s, d.max(axis=1), rtol=1e-15)
    with pytest.raises(g.GlamerError):
        gpu_knn(x, y, 65)
    with pytest.raises(g.GlamerError):
        gpu_knn(np.zeros(200), np.arange(200.0), 0)


# ---------------------------------------------------------------- glm_knn
# raw positions in 2D or 3D, optionally per species (bounding-box hierarchy)

def gpu_knn_pos(x, y, k, z=None, species=None):
    import paper_1312_1128_amd as g
    import torch

    sp = torch.from_numpy(np.ascontiguousarray(species, dtype=np.int32)).cuda() if species is not None else None
    s = g.knn(dev(x), dev(y), k, z=dev(z) if z is not None else None, species=sp)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def clustered_3d(n, seed):
    x, y = clustered(n, seed)
    g = synth.rng(seed + 1)
    z = np.concatenate([g.uniform(-1, 1, n // 2), g.normal(0.1, 1e-3, n // 4), g.normal(0, 5, n - n // 2 - n // 4)])
    z[10:30] = z[3]  # the 21 coincident particles stay coincident in space
    x[40], y[40] = x[41], y[41]  # same projection, apart in z
    return x, y, z


@pytest.mark.parametrize("k", [1, 8, 16, 32, 33, 64])
def test_knn_positions_3d_and_2d_match_oracle(ora, k):
    x, y, z = clustered_3d(9001, 87)
    say(f"[gpu] glm_knn n={x.size} k={k} (3D and 2D)")
    got3 = gpu_knn_pos(x, y, k, z=z)
    np.testing.assert_array_max_ulp(got3, ora.knn(x, y, k, z=z), maxulp=1)
    got2 = gpu_knn_pos(x, y, k)
    np.testing.assert_array_max_ulp(got2, ora.knn(x, y, k), maxulp=1)
    # the quad-tree search gives the same 2D lengths
    np.testing.assert_array_max_ulp(got2, gpu_knn(x, y, k), maxulp=1)
    if k <= 20:
        assert np.all(got3[[3] + list(range(10, 30))] == 0.0)
    if k == 1:
        assert got2[40] == 0.0 and got3[40] > 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_knn_positions_per_species(ora, dim):
    g0 = synth.rng(89 + dim)
    x, y, z = clustered_3d(12_000, 91)
    zz = z if dim == 3 else None
    # a large species, a rare one spread over everything, one with exactly k + 1
    # members, and 40 small ones: 43 segments
    sp = np.where(g0.random(x.size) < 0.05, 1000, 0).astype(np.int32)
    sp[100:133] = 5  # 33 = k + 1 members for k = 32
    for t in range(40):
        sp[200 + 60 * t: 200 + 60 * t + 50] = 2000 + t
    say(f"[gpu] glm_knn per species, {dim}D, {np.unique(sp).size} species")
    for k in (16, 32):
        got = gpu_knn_pos(x, y, k, z=zz, species=sp)
        np.testing.assert_array_max_ulp(got, ora.knn(x, y, k, z=zz, species=sp), maxulp=1)
    # one label for everybody is no species at all
    np.testing.assert_array_equal(gpu_knn_pos(x, y, 8, z=zz, species=np.full(x.size, 7)),
                                  gpu_knn_pos(x, y, 8, z=zz))


def test_knn_positions_nfw_3d_sampled(ora):
    """3D smoothing of a 1e6-particle NFW halo (the positions before
    projection): sampled particles against the brute force."""
    x, y, z = synth.nfw_3d(1_000_000, synth.BASE_SEED + 2)
    say("[gpu] glm_knn 3D nfw n=1e6")
    got = gpu_knn_pos(x, y, 32, z=z)
    at = synth.sample_rays(x, y, 2048, 93)
    np.testing.assert_array_max_ulp(got[at], ora.knn(x, y, 32, at=at, z=z), maxulp=1)
    # 3D neighbours are never nearer than projected ones
    assert np.all(got >= gpu_knn_pos(x, y, 32))


def test_knn_positions_invalid():
    import paper_1312_1128_amd as g

    g0 = synth.rng(95)
    x, y, z = g0.uniform(size=300), g0.uniform(size=300), g0.uniform(size=300)
    np.testing.assert_array_equal(gpu_knn_pos(np.array([0.0, 3.0]), np.array([0.0, 4.0]), 1, z=np.array([0.0, 12.0])),
                                  [13.0, 13.0])
    with pytest.raises(g.GlamerError, match="k must"):
        gpu_knn_pos(x, y, 65, z=z)
    sp = np.zeros(300, np.int32)
    sp[:8] = 3  # 8 particles: no 8th neighbour among them
    with pytest.raises(g.GlamerError, match="species"):
        gpu_knn_pos(x, y, 8, z=z, species=sp)
    sp[:8] = 70000
    with pytest.raises(g.GlamerError, match="species id"):
        gpu_knn_pos(x, y, 4, z=z, species=sp)
    z2 = z.copy()
    z2[17] = np.nan
    with pytest.raises(g.GlamerError, match="NaN"):
        gpu_knn_pos(x, y, 4, z=z2)
