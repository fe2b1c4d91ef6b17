"""Seeded random configurations of the whole path against oracle B (the FP64
reference tree with the same decisions): particle layouts (uniform, clustered,
coincident, collinear), kinds (Gaussians with some point masses, NFW halos),
theta, leaf size, order and cutoff drawn at random; rays uniform over and
around the particles plus rays exactly on particles.  Per ray the interaction
counts must be identical and alpha, kappa, gamma and the potential equal to
FP32 rounding; the adjoint (random cotangents, rays off the particles) must
match the oracle's frozen-tree gradient.

GLM_RANDOM_SEEDS=a:b runs seeds a .. b-1 instead of the default 0 .. 47.  Of
seeds 0 .. 1447 one misses: seed 203 (NFW halos up to 0.3 across, collinear,
leaf size 1), where one particle's adjoint component is 2.6 times outside the
bound, the FP32 halo terms summed over the rays with cancellation.  Of seeds
1448 .. 6447 four miss, all lenses of 2 or 3 heavily overlapping particles:
2119 and 6030 on the shear (a ray inside a big particle's support whose box
is expanded, where the FP32 point part m / r^2 cancels against the list's
Gaussian - point term), 5786 and 5804 on the adjoint (terms cancelling over
the rays, as in seed 203).  Seeds 6448 .. 16447 miss 7 times, by 1.1 to 13.5
times the bound, on the shear of the same cancellation near halo cores."""
import os

import numpy as np
import pytest

import synth
from gpu_helpers import assert_matches_oracle_tree, build, dev, say, shoot

pytestmark = pytest.mark.gpu

SEEDS = range(*(int(v) for v in os.environ.get("GLM_RANDOM_SEEDS", "0:48").split(":")))


def make_case(seed):
    g = synth.rng(9000 + seed)
    n = int(round(10 ** g.uniform(0, 3.5)))
    layout = ["uniform", "clustered", "coincident", "collinear"][seed % 4]
    if layout == "uniform":
        x, y = g.uniform(-0.5, 0.5, n), g.uniform(-0.5, 0.5, n)
    elif layout == "clustered":
        c = g.uniform(-0.4, 0.4, (5, 2))
        k = g.integers(0, 5, n)
        x, y = c[k, 0] + 0.02 * g.normal(size=n), c[k, 1] + 0.02 * g.normal(size=n)
    elif layout == "coincident":
        x, y = g.uniform(-0.5, 0.5, n), g.uniform(-0.5, 0.5, n)
        dup = g.random(n) < 0.3
        x[dup], y[dup] = x[0], y[0]
    else:
        t = g.uniform(-0.5, 0.5, n)
        x, y = t, 0.3 * t + 1e-3 * g.normal(size=n)
    m = g.uniform(0.1, 1.0, n) / n
    nfw = seed % 3 == 2
    if nfw:
        s = g.uniform(0.0, 0.3, n)
        q = float(g.uniform(2.0, 8.0))  # concentration
    else:
        s = g.uniform(0.002, 0.1, n)
        s[g.random(n) < 0.2] = 0.0
        q = float(g.uniform(1.0, 5.0))
    lens = synth.Lens(x, y, m, s, q=q)
    theta = float(g.uniform(0.0, 0.58))
    leaf = int(g.integers(1, 65))
    order = int(g.integers(0, 13))
    nr = 300
    lo, hi = min(x.min(), y.min()) - 0.1, max(x.max(), y.max()) + 0.1
    rx, ry = g.uniform(lo, hi, nr), g.uniform(lo, hi, nr)
    on = g.integers(0, n, 10)
    rx, ry = np.concatenate([rx, x[on]]), np.concatenate([ry, y[on]])
    return lens, nfw, theta, leaf, order, rx, ry


@pytest.mark.parametrize("seed", SEEDS)
def test_random_configuration_matches_oracle_tree(ora, seed):
    from paper_1312_1128_amd import GLM_NFW_HALOS

    lens, nfw, theta, leaf, order, rx, ry = make_case(seed)
    say(f"[gpu] random config {seed}: n={lens.n} nfw={nfw} theta={theta:.3f} L={leaf} p={order} q={lens.q:.2f}")
    tree = build(lens, theta, leaf, order, flags=GLM_NFW_HALOS if nfw else 0)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order, nfw=nfw)
    ref, rcnt = T.shoot(rx, ry, counts=True)
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    assert_matches_oracle_tree(got, ref)
    # potential
    import paper_1312_1128_amd as g
    import torch

    o = g.shoot_potential(tree, dev(rx), dev(ry))
    torch.cuda.synchronize()
    psi = o["psi"].double().cpu().numpy()
    psi_ref = T.shoot_psi(rx, ry)
    assert np.abs(psi - psi_ref).max() <= 2e-6 * np.abs(psi_ref).max()
    # adjoint with random cotangents of alpha, on the rays off the particles
    nr = rx.size - 10
    ga = synth.rng(9500 + seed).normal(size=(nr, 2)).astype(np.float32).astype(np.float64)
    t = torch.from_numpy(np.ascontiguousarray(ga, dtype=np.float32)).cuda()
    grads = g.shoot_adjoint(tree, dev(rx[:nr]), dev(ry[:nr]), t[:, 0].contiguous(), t[:, 1].contiguous())
    torch.cuda.synchronize()
    refs = T.grad(rx[:nr], ry[:nr], ga)
    for name, a, b in zip("mxys", grads, refs):
        a = a.cpu().numpy()
        sc = np.abs(b).max()
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 2e-6 * sc), name
