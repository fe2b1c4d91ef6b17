"""Lensing potential and time delay on the GPU (Sec. 3.2: alpha = grad psi,
time delay |alpha|^2 / 2 - psi) against the FP64 oracle tree (same
decisions) and the FP64 brute force."""
import numpy as np
import pytest

import synth
from gpu_helpers import build, dev, say, shoot

pytestmark = pytest.mark.gpu


def mixed_lens(n, seed):
    lens = synth.gaussian_blobs(n, seed, s_lo=0.003, s_hi=0.3)
    lens.s[synth.rng(seed + 1).random(n) < 0.2] = 0.0
    return lens


def gpu_potential(tree, rx, ry):
    import paper_1312_1128_amd as g
    import torch

    o = g.shoot_potential(tree, dev(rx), dev(ry))
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in o.items()}


CASES = {
    "point_masses_1k": (lambda: synth.point_masses(1000, synth.BASE_SEED + 1), 0.5, 8, 2),
    "mixed_3k_leaf3": (lambda: mixed_lens(3000, 17), 0.5, 3, 4),
    "nfw_20k": (lambda: synth.nfw_halo(20000, synth.BASE_SEED + 3), 0.3, 16, 8),
}


@pytest.mark.parametrize("case", list(CASES))
def test_potential_matches_oracle_tree(ora, case):
    make, theta, leaf, order = CASES[case]
    lens = make()
    say(f"[gpu] potential {case}: n={lens.n}")
    tree = build(lens, theta, leaf, order)
    rx, ry = synth.ray_grid(67)
    got = gpu_potential(tree, rx, ry)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order)
    ref = T.shoot_psi(rx, ry)
    err = np.abs(got["psi"] - ref) / np.abs(ref).max()
    say(f"  psi vs oracle tree: max {err.max():.2e} (relative to max |psi|)")
    assert err.max() < 2e-6
    # the deflection of this walk is the alpha-only walk's (a small shoot
    # splits the box array over several wavefronts: sums regrouped only)
    a = shoot(tree, rx, ry, alpha_only=True)
    np.testing.assert_allclose(got["a1"], a[:, 0], rtol=2e-6, atol=1e-7 * np.abs(a[:, 0]).max())
    np.testing.assert_allclose(got["a2"], a[:, 1], rtol=2e-6, atol=1e-7 * np.abs(a[:, 1]).max())
    td = 0.5 * (got["a1"] ** 2 + got["a2"] ** 2) - got["psi"]
    np.testing.assert_allclose(got["tdelay"], td, rtol=1e-5, atol=1e-6 * np.abs(td).max())


def test_potential_theta_zero_and_bruteforce(ora):
    lens = mixed_lens(4000, 23)
    rx, ry = synth.uniform_points(1000, 24)
    ref = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry)
    got = gpu_potential(build(lens, 0.0, 8, 2), rx, ry)
    assert np.abs(got["psi"] - ref).max() / np.abs(ref).max() < 2e-6
    # the smoothed NFW halo at the headline settings, against the brute force
    halo = synth.nfw_halo(100_000, synth.BASE_SEED + 5)
    hx, hy = synth.ray_grid(64)
    got = gpu_potential(build(halo, 0.3, 16, 8), hx, hy)
    ref = ora.direct_psi(halo.x, halo.y, halo.m, halo.s, halo.q, hx, hy)
    err = np.abs(got["psi"] - ref) / np.abs(ref)
    say(f"[gpu] potential nfw 1e5 vs brute force: max rel {err.max():.2e}")
    assert err.max() < 1e-5
