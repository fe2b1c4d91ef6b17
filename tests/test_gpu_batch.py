"""Batched walks, device refinement rounds (and their HIP-graph replay) and the
autotuner, against per-lens walks, the oracle's statement of the refinement
rule (oracle/refine.py), and the FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import build, dev, rel_err, say, shoot, stats

pytestmark = pytest.mark.gpu


def to_np(out, names=("a1", "a2", "kappa", "g1", "g2")):
    return np.stack([out[k].double().cpu().numpy() for k in names], axis=1)


def test_batched_equals_per_lens_and_oracle(ora):
    import paper_1312_1128_amd as g
    import torch

    lenses = synth.workload_batched_lenses(nlens=10, seed=401, scale=0.05)
    lenses[3] = (lenses[3][0], np.zeros(0), np.zeros(0))           # a lens without rays
    lenses[5] = (lenses[5][0], lenses[5][1][:1], lenses[5][2][:1])  # a single ray
    say(f"[gpu] batched: {[(l.n, rx.size) for l, rx, _ in lenses]}")
    trees = [build(l, 0.3, 8, 8) for l, _, _ in lenses]
    rays = [(dev(rx), dev(ry)) for _, rx, ry in lenses]
    outs = g.shoot_batched(trees, rays)
    torch.cuda.synchronize()
    for (l, rx, ry), t, o in zip(lenses, trees, outs):
        if rx.size == 0:
            continue
        got = to_np(o)
        # the same per-ray decisions; a single small walk may split the box
        # array over several wavefronts, which only regroups the FP32 sums
        single, cnt = shoot(t, rx, ry, counts=True)
        np.testing.assert_allclose(got[:, :2], single[:, :2], rtol=2e-6, atol=1e-7 * np.abs(single[:, :2]).max())
        np.testing.assert_allclose(got[:, 2], single[:, 2], rtol=2e-6, atol=1e-7 * np.abs(single[:, 2]).max())
        np.testing.assert_allclose(got[:, 3:], single[:, 3:], rtol=1e-5, atol=1e-6 * np.abs(single[:, 3:]).max())
        idx = synth.sample_rays(rx, ry, 128, 5)
        ref = ora.direct(l.x, l.y, l.m, l.s, l.q, rx[idx], ry[idx])
        ea, ek, eg = rel_err(got[idx], ref)
        assert ea.max() <= 1e-4 and ek.max() <= 1e-4 and eg.max() <= 1e-4
    # alpha only
    outa = g.shoot_batched(trees, rays, alpha_only=True)
    for o, oa in zip(outs, outa):
        np.testing.assert_array_equal(o["a1"].cpu().numpy(), oa["a1"].cpu().numpy())


def test_refine_round_matches_rule():
    import paper_1312_1128_amd as g
    import torch

    say("[gpu] refine round")
    gen = synth.rng(411)
    n, k = 5000, 517
    cap = n + 8 * k
    cx = np.zeros(cap)
    cy = np.zeros(cap)
    side = np.zeros(cap)
    cx[:n], cy[:n] = gen.uniform(-1, 1, n), gen.uniform(-1, 1, n)
    side[:n] = gen.choice([0.01, 0.02, 0.03], n)
    kap = gen.normal(size=cap).astype(np.float32)
    g1 = gen.normal(size=cap).astype(np.float32)
    g2 = gen.normal(size=cap).astype(np.float32)
    kap[100:110] = kap[50]  # ties
    g1[100:110] = g1[50]
    g2[100:110] = g2[50]
    side[100:110] = side[50]
    tx, ty, ts = dev(cx), dev(cy), dev(side)
    f = lambda a: torch.from_numpy(a).cuda()
    refined = torch.zeros(k, dtype=torch.int32, device="cuda")
    g.refine_round(tx, ty, ts, f(kap), f(g1), f(g2), n, k, refined=refined)
    torch.cuda.synchronize()
    from oracle import refine

    ex, ey, es = cx.copy(), cy.copy(), side.copy()
    order = refine.refine_round(ex, ey, es, kap, g1, g2, n, k)
    np.testing.assert_array_equal(refined.cpu().numpy(), order)
    np.testing.assert_array_equal(tx.cpu().numpy(), ex)
    np.testing.assert_array_equal(ty.cpu().numpy(), ey)
    np.testing.assert_array_equal(ts.cpu().numpy(), es)


def small_microlensing():
    halo = synth.nfw_halo(100_000, 421)
    stars = synth.star_patch(10_000, 423)
    lens = synth.Lens(np.concatenate([halo.x, stars.x]), np.concatenate([halo.y, stars.y]),
                      np.concatenate([halo.m, stars.m]), np.concatenate([halo.s, stars.s]))
    cx, cy = synth.ray_grid(64, -0.005, 0.005)
    return lens, cx + 0.25, cy, np.full(64 * 64, 0.01 / 64)


def test_refinement_rounds_graph_replay_and_oracle(ora):
    import paper_1312_1128_amd as g
    import torch

    lens, cx, cy, side = small_microlensing()
    say(f"[gpu] refinement rounds: n={lens.n}")
    tree = build(lens, 0.3, 8, 8)
    sched = g.refine_schedule(cx.size, rounds=4)
    run = g.RefinementRun(tree, dev(cx), dev(cy), dev(side), sched)
    n = run.run()
    torch.cuda.synchronize()
    eager = {k: v[:n].cpu().numpy().copy() for k, v in run.out.items()}
    ex = run.cx[:n].cpu().numpy().copy()
    # every round's rays against the FP64 brute force
    a = 0
    for r, size in enumerate(run.sizes):
        idx = a + synth.sample_rays(np.zeros(size), None, 256, 430 + r)
        ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, ex[idx], run.cy[:n].cpu().numpy()[idx])
        got = np.stack([eager[k][idx] for k in ["a1", "a2", "kappa", "g1", "g2"]], axis=1).astype(np.float64)
        ea, ek, eg = rel_err(got, ref)
        ok = np.abs(ref[:, 2]) > 0
        assert ea.max() <= 1e-4 and eg.max() <= 1e-4 and np.all(ek[ok] <= 1e-4), r
        a += size
    # the whole schedule as one HIP graph, replayed with eager work in between
    graph = run.capture()
    for rep in range(3):
        for v in run.out.values():
            v.zero_()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(run.cx[:n].cpu().numpy(), ex)
        for k, v in run.out.items():
            np.testing.assert_array_equal(v[:n].cpu().numpy(), eager[k])
        g.shoot(tree, dev(cx[:100]), dev(cy[:100]))  # unrelated eager work between replays
        torch.cuda.synchronize()


def test_autotune_picks_a_passing_configuration(ora):
    """The tuner accepts a configuration on 16,384 random rays plus the 4,096
    nearest the densest point; the choice must then hold on held-out rays
    against the CPU brute force, and be the fastest accepted row."""
    import paper_1312_1128_amd as g

    lens = synth.nfw_halo(50_000, 441)
    rx, ry = synth.ray_grid(256)
    say("[gpu] autotune")
    X, Y, M, S, RX, RY = (dev(a) for a in (lens.x, lens.y, lens.m, lens.s, rx, ry))
    best, table = g.autotune(X, Y, M, S, RX, RY, thetas=(0.3, 0.5), orders=(4, 6, 8, 10), leaves=(8, 16), reps=2)
    assert best is not None and best["err"] <= 1e-4 and best["rays_checked"] >= 16384
    # held out: rays not in the tuner's validation set, against the FP64 brute force
    val = set(g.batch.validation_rays(X, Y, S, RX, RY).cpu().numpy().tolist())
    rest = np.array(sorted(set(range(rx.size)) - val))
    hold = rest[synth.sample_rays(rest, None, 4096, 443)]
    tree = build(lens, best["theta"], best["leaf_size"], best["order"])
    got = shoot(tree, rx[hold], ry[hold])
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx[hold], ry[hold])
    ea, ek, eg = rel_err(got, ref)
    ok = ref[:, 2] != 0
    say(f"  chosen {best['theta']}, {best['order']}, {best['leaf_size']}: held-out max e_alpha {ea.max():.2e} "
        f"e_kappa {ek[ok].max():.2e} e_gamma {eg.max():.2e}")
    assert ea.max() <= 1e-4 and eg.max() <= 1e-4 and np.all(ek[ok] <= 1e-4)
    # every accepted row met the tolerance, every refused one missed it
    for t in table:
        err = max(t["err_alpha"], t["err_kappa"], t["err_gamma"])
        assert t["ok"] == (err <= 1e-4), t
    passing = [t for t in table if t["ok"]]
    assert best["ms"] == min(t["ms"] for t in passing)
