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
