"""GPU adjoint walk (glm_shoot_adjoint through the C ABI) against the CPU
oracle: the oracle tree's FP64 adjoint on the same tree and cotangents (itself
pinned by frozen-walk finite differences on the CPU), the FP64 brute-force
gradient, and exact identities of the lensing sums."""
import numpy as np
import pytest

import synth
from gpu_helpers import build, dev, say, shoot

pytestmark = pytest.mark.gpu


def gpu_grad(tree, rx, ry, ga):
    import paper_1312_1128_amd as g
    import torch

    t = torch.from_numpy(np.ascontiguousarray(ga, dtype=np.float32)).cuda()
    out = g.shoot_adjoint(tree, dev(rx), dev(ry), t[:, 0].contiguous(), t[:, 1].contiguous())
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def compare(name, got, ref, rtol, scale_frac):
    sc = np.abs(ref).max()
    err = np.abs(got - ref)
    bad = err > rtol * np.abs(ref) + scale_frac * sc
    say(f"  {name}: max |err|/max|ref| {err.max() / sc:.3e}, bad {bad.sum()}")
    assert not bad.any(), name


def mixed_lens(n, seed):
    lens = synth.gaussian_blobs(n, seed, s_lo=0.003, s_hi=0.3)
    g = synth.rng(seed + 1)
    lens.s[g.random(n) < 0.2] = 0.0
    return lens


@pytest.mark.parametrize("case", ["mixed_3k", "nfw_20k", "point_masses_2k", "clump_100"])
def test_adjoint_matches_oracle_tree(ora, case):
    if case == "mixed_3k":
        lens, theta, leaf, order = mixed_lens(3000, 301), 0.5, 4, 4
    elif case == "clump_100":
        # 100 coincident particles: one leaf at the depth cap holding more than
        # a wavefront's worth of particles
        lens, theta, leaf, order = mixed_lens(1000, 311), 0.5, 8, 4
        lens.x[:100], lens.y[:100] = lens.x[0], lens.y[0]
    elif case == "nfw_20k":
        lens, theta, leaf, order = synth.nfw_halo(20000, 303), 0.3, 8, 8
    else:
        lens, theta, leaf, order = synth.point_masses(2000, 305), 0.5, 8, 3
    say(f"[gpu] adjoint {case}: n={lens.n} theta={theta} p={order}")
    rx, ry = synth.uniform_points(3000, 307)
    ga = synth.rng(309).normal(size=(rx.size, 2)).astype(np.float32).astype(np.float64)
    tree = build(lens, theta, leaf, order)
    dm, dx, dy, ds = gpu_grad(tree, rx, ry, ga)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order)
    rm, rxg, ryg, rs = T.grad(rx, ry, ga)
    compare("dL/dm", dm, rm, 1e-4, 2e-6)
    compare("dL/dx", dx, rxg, 1e-4, 2e-6)
    compare("dL/dy", dy, ryg, 1e-4, 2e-6)
    compare("dL/ds", ds, rs, 1e-4, 2e-6)


def test_adjoint_fitting_workload_vs_bruteforce(ora):
    """1e5 smoothed NFW particles, 1e5 rays uniform in [-0.5, 0.5]^2; target
    source positions beta* = x - alpha_true + N(0, 1e-4); L = sum |x - alpha -
    beta*|^2, so dL/dalpha = -2 (x - alpha - beta*).  Tree theta = 0.3, p = 8."""
    lens = synth.nfw_halo(100_000, synth.BASE_SEED + 5)
    rx, ry = synth.uniform_points(100_000, synth.BASE_SEED + 6)
    say(f"[gpu] adjoint fitting workload n={lens.n} rays={rx.size}")
    a_true = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry)[:, :2]
    noise = synth.rng(synth.BASE_SEED + 8).normal(0.0, 1e-4, size=(rx.size, 2))
    bx, by = rx - a_true[:, 0] + noise[:, 0], ry - a_true[:, 1] + noise[:, 1]
    # the cotangents come from the oracle tree's forward (an FP32 input to both sides)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.3, 8, 8)
    AB = T.shoot(rx, ry)
    ga = np.stack([-2 * (rx - AB[:, 0] - bx), -2 * (ry - AB[:, 1] - by)], axis=1)
    ga = ga.astype(np.float32).astype(np.float64)
    tree = build(lens, 0.3, 8, 8)
    A = shoot(tree, rx, ry)
    dm, dx, dy, ds = gpu_grad(tree, rx, ry, ga)
    # the same tree in FP64 (decisions identical to the GPU walk)
    rm, rxg, ryg, rs = T.grad(rx, ry, ga)
    compare("tree dL/dm", dm, rm, 1e-4, 2e-6)
    compare("tree dL/dx", dx, rxg, 1e-4, 2e-6)
    compare("tree dL/dy", dy, ryg, 1e-4, 2e-6)
    compare("tree dL/ds", ds, rs, 1e-4, 2e-6)
    # brute force: the tree's Jacobian is an approximation at the 1e-5 level
    bm, bxg, byg, bs = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry, ga)
    for nm, a, b in [("m", dm, bm), ("x", dx, bxg), ("y", dy, byg), ("s", ds, bs)]:
        e = np.abs(a - b).max() / np.abs(b).max()
        say(f"  brute-force dL/d{nm}: max |err| / max |grad| = {e:.3e}")
        assert e < 1e-3
    # Euler: alpha is homogeneous of degree 1 in the masses
    L1 = np.sum(ga[:, 0] * A[:, 0] + ga[:, 1] * A[:, 1])
    assert abs(np.sum(lens.m * dm) - L1) <= 1e-4 * np.sum(np.abs(lens.m * dm))


def test_adjoint_headline_1e6_vs_oracle_tree(ora):
    """The adjoint at the headline size: 1e6 smoothed NFW particles, theta =
    0.3, p = 8, leaf size 16, on 4,096 seeded rays of the 2048^2 grid plus the
    512 nearest the halo centre, with the fitting loss L = sum |x - alpha -
    beta*|^2 (beta* = x - alpha_true + N(0, 1e-4), alpha_true from the FP64
    brute force), against the oracle tree's frozen-walk gradient."""
    lens, gx, gy = synth.workload_nfw()
    central = np.argsort(gx * gx + gy * gy, kind="stable")[:512]
    idx = np.union1d(synth.sample_rays(gx, gy, 4096, synth.BASE_SEED + 12), central)
    rx, ry = gx[idx], gy[idx]
    say(f"[gpu] adjoint at 1e6 particles: {rx.size} rays")
    a_true = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry)[:, :2]
    noise = synth.rng(synth.BASE_SEED + 13).normal(0.0, 1e-4, size=(rx.size, 2))
    bx, by = rx - a_true[:, 0] + noise[:, 0], ry - a_true[:, 1] + noise[:, 1]
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.3, 16, 8)
    AB = T.shoot(rx, ry)
    ga = np.stack([-2 * (rx - AB[:, 0] - bx), -2 * (ry - AB[:, 1] - by)], axis=1)
    ga = ga.astype(np.float32).astype(np.float64)
    tree = build(lens, 0.3, 16, 8)
    dm, dx, dy, ds = gpu_grad(tree, rx, ry, ga)
    rm, rxg, ryg, rs = T.grad(rx, ry, ga)
    compare("dL/dm", dm, rm, 1e-4, 2e-6)
    compare("dL/dx", dx, rxg, 1e-4, 2e-6)
    compare("dL/dy", dy, ryg, 1e-4, 2e-6)
    compare("dL/ds", ds, rs, 1e-4, 2e-6)
    # Euler: sum_i m_i dL/dm_i = sum_r ga . alpha_r (alpha is linear in the masses)
    A = shoot(tree, rx, ry)
    L1 = np.sum(ga[:, 0] * A[:, 0] + ga[:, 1] * A[:, 1])
    assert abs(np.sum(lens.m * dm) - L1) <= 1e-5 * np.sum(np.abs(lens.m * dm))


def test_adjoint_workspace_and_concurrent_streams(ora):
    """The adjoint only reads the tree: two adjoints of one tree on two streams
    with their own workspaces give the sequential result (to the rounding of
    the FP64 atomics); a workspace below glm_adjoint_workspace_bytes is refused."""
    import paper_1312_1128_amd as g
    import torch

    lens = synth.nfw_halo(30000, 341)
    rx, ry = synth.uniform_points(20000, 343)
    say("[gpu] adjoint workspaces on two streams")
    tree = build(lens, 0.3, 8, 6)
    gen = synth.rng(345)
    cots = [torch.from_numpy(gen.normal(size=rx.size).astype(np.float32)).cuda() for _ in range(4)]
    X, Y = dev(rx), dev(ry)
    seq = [g.shoot_adjoint(tree, X, Y, cots[2 * j], cots[2 * j + 1]) for j in range(2)]
    torch.cuda.synchronize()
    need = g.adjoint_workspace_bytes(tree, rx.size)
    assert need > g.workspace_bytes(rx.size)
    with pytest.raises(g.GlamerError) as e:
        g.shoot_adjoint(tree, X, Y, cots[0], cots[1],
                        workspace=torch.empty(need - 8, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -2
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [torch.empty(need, dtype=torch.uint8, device="cuda") for _ in range(2)]
    outs = []
    torch.cuda.synchronize()
    for j, st in enumerate(streams):
        with torch.cuda.stream(st):
            outs.append(g.shoot_adjoint(tree, X, Y, cots[2 * j], cots[2 * j + 1], workspace=wss[j]))
    torch.cuda.synchronize()
    for j in range(2):
        for a, b in zip(outs[j], seq[j]):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max())


def test_adjoint_identities_and_autograd(ora):
    import paper_1312_1128_amd as g
    import torch

    lens = mixed_lens(4000, 311)
    rx, ry = synth.uniform_points(2000, 313)
    say("[gpu] adjoint identities + autograd")
    ga = synth.rng(315).normal(size=(rx.size, 2)).astype(np.float32).astype(np.float64)
    tree = build(lens, 0.5, 8, 5)
    B = shoot(tree, rx, ry)
    dm, dx, dy, ds = gpu_grad(tree, rx, ry, ga)
    L1 = np.sum(ga[:, 0] * B[:, 0] + ga[:, 1] * B[:, 1])
    assert abs(np.sum(lens.m * dm) - L1) <= 1e-4 * np.sum(np.abs(lens.m * dm))
    k, g1, g2 = B[:, 2], B[:, 3], B[:, 4]
    tx = -np.sum((k + g1) * ga[:, 0] + g2 * ga[:, 1])
    ty = -np.sum(g2 * ga[:, 0] + (k - g1) * ga[:, 1])
    sc = np.sum(np.abs(dx)) + np.sum(np.abs(dy))
    assert abs(np.sum(dx) - tx) <= 1e-4 * sc and abs(np.sum(dy) - ty) <= 1e-4 * sc
    # the autograd wrapper gives the same gradient
    m_t = dev(lens.m).requires_grad_(True)
    x_t = dev(lens.x).requires_grad_(True)
    y_t = dev(lens.y).requires_grad_(True)
    s_t = dev(lens.s).requires_grad_(True)
    a1, a2 = g.ShootFn.apply(dev(rx), dev(ry), m_t, x_t, y_t, s_t,
                             dict(theta=0.5, q=lens.q, leaf_size=8, order=5))
    gt = torch.from_numpy(ga.astype(np.float32)).cuda()
    (a1 * gt[:, 0] + a2 * gt[:, 1]).sum().backward()
    np.testing.assert_allclose(m_t.grad.cpu().numpy(), dm, rtol=1e-6, atol=1e-9 * np.abs(dm).max())
    np.testing.assert_allclose(x_t.grad.cpu().numpy(), dx, rtol=1e-6, atol=1e-9 * np.abs(dx).max())
    np.testing.assert_allclose(s_t.grad.cpu().numpy(), ds, rtol=1e-6, atol=1e-9 * np.abs(ds).max())


# ------------------------------------------------ kappa and gamma cotangents

def gpu_grad_kg(tree, rx, ry, ga, gk, gg):
    import paper_1312_1128_amd as g
    import torch

    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() if a is not None else None
    out = g.shoot_adjoint(tree, dev(rx), dev(ry), f(ga[:, 0]) if ga is not None else None,
                          f(ga[:, 1]) if ga is not None else None, gk=f(gk), gg1=f(gg[:, 0]), gg2=f(gg[:, 1]))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("case", ["mixed_3k", "nfw_20k", "point_masses_2k"])
def test_adjoint_kappa_gamma_matches_oracle_tree(ora, case):
    """L = sum_r ga . alpha + gk kappa + gg . gamma: the gamma cotangent
    reaches the box moments (gamma of a box is the derivative of its alpha
    series), the kappa one only the direct terms."""
    if case == "mixed_3k":
        lens, theta, leaf, order = mixed_lens(3000, 311), 0.5, 4, 4
    elif case == "nfw_20k":
        lens, theta, leaf, order = synth.nfw_halo(20000, 313), 0.3, 8, 8
    else:
        lens, theta, leaf, order = synth.point_masses(2000, 315), 0.5, 8, 3
    say(f"[gpu] adjoint with kappa, gamma cotangents {case}: n={lens.n} theta={theta} p={order}")
    rx, ry = synth.uniform_points(3000, 317)
    g0 = synth.rng(319)
    ga, gk, gg = f32(g0.normal(size=(rx.size, 2))), f32(g0.normal(size=rx.size)), f32(g0.normal(size=(rx.size, 2)))
    tree = build(lens, theta, leaf, order)
    got = gpu_grad_kg(tree, rx, ry, ga, gk, gg)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order)
    ref = T.grad(rx, ry, ga, gk=gk, gg=gg)
    for name, a, b in zip(["dL/dm", "dL/dx", "dL/dy", "dL/ds"], got, ref):
        compare(name, a, b, 1e-4, 2e-6)
    # kappa and gamma cotangents alone (no alpha cotangent at all)
    got = gpu_grad_kg(tree, rx, ry, None, gk, gg)
    ref = T.grad(rx, ry, 0 * ga, gk=gk, gg=gg)
    for name, a, b in zip(["kg dL/dm", "kg dL/dx", "kg dL/dy", "kg dL/ds"], got, ref):
        compare(name, a, b, 1e-4, 2e-6)


@pytest.mark.parametrize("order", range(13))
def test_adjoint_every_order_matches_oracle_tree(ora, order):
    """Every multipole order the boundary accepts, with alpha cotangents and with
    kappa and gamma ones: an accepted box's 2p + 4 adjoint words are summed over
    the wavefront's lanes in registers, in a lane layout that depends on the
    number of words (odd and even halves, every count from 4 to 28)."""
    lens = mixed_lens(1500, 331)
    theta, leaf = 0.6, 8
    say(f"[gpu] adjoint at order {order}: n={lens.n} theta={theta}")
    rx, ry = synth.uniform_points(1500, 333)
    g0 = synth.rng(335 + order)
    ga, gk, gg = f32(g0.normal(size=(rx.size, 2))), f32(g0.normal(size=rx.size)), f32(g0.normal(size=(rx.size, 2)))
    tree = build(lens, theta, leaf, order)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order)
    for name, a, b in zip(["dL/dm", "dL/dx", "dL/dy", "dL/ds"], gpu_grad(tree, rx, ry, ga), T.grad(rx, ry, ga)):
        compare(name, a, b, 1e-4, 2e-6)
    got = gpu_grad_kg(tree, rx, ry, ga, gk, gg)
    ref = T.grad(rx, ry, ga, gk=gk, gg=gg)
    for name, a, b in zip(["kg dL/dm", "kg dL/dx", "kg dL/dy", "kg dL/ds"], got, ref):
        compare(name, a, b, 1e-4, 2e-6)


def test_adjoint_kappa_gamma_theta_zero_vs_bruteforce(ora):
    lens = mixed_lens(2500, 321)
    rx, ry = synth.uniform_points(1500, 323)
    g0 = synth.rng(325)
    ga, gk, gg = f32(g0.normal(size=(rx.size, 2))), f32(g0.normal(size=rx.size)), f32(g0.normal(size=(rx.size, 2)))
    say("[gpu] adjoint with kappa, gamma cotangents, theta = 0 vs the FP64 brute-force gradient")
    got = gpu_grad_kg(build(lens, 0.0, 8, 2), rx, ry, ga, gk, gg)
    ref = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry, ga, gk=gk, gg=gg)
    for name, a, b in zip(["dL/dm", "dL/dx", "dL/dy", "dL/ds"], got, ref):
        compare(name, a, b, 1e-4, 2e-6)


def test_shootfn_lensing_outputs_autograd():
    """ShootFn with lensing=True returns alpha, kappa, gamma; its backward is
    the adjoint walk with all five cotangents."""
    import paper_1312_1128_amd as g
    import torch

    lens = mixed_lens(2000, 331)
    rx, ry = synth.uniform_points(800, 333)
    x, y, m, s = (dev(a).requires_grad_(True) for a in (lens.x, lens.y, lens.m, lens.s))
    params = dict(theta=0.5, q=lens.q, leaf_size=8, order=4)
    outs = g.ShootFn.apply(dev(rx), dev(ry), m, x, y, s, params, True)
    assert len(outs) == 5
    w = [torch.from_numpy(synth.rng(335 + i).normal(size=rx.size).astype(np.float32)).cuda() for i in range(5)]
    loss = sum((o * wi).sum() for o, wi in zip(outs, w))
    loss.backward()
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), **params)
    ref = g.shoot_adjoint(tree, dev(rx), dev(ry), w[0], w[1], gk=w[2], gg1=w[3], gg2=w[4])
    torch.cuda.synchronize()
    for t, r in zip([m, x, y, s], ref):
        np.testing.assert_allclose(t.grad.cpu().numpy(), r.cpu().numpy(), rtol=1e-6, atol=1e-9 * float(r.abs().max()))
