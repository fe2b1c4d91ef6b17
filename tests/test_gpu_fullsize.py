"""The benchmark's secondary workloads at their full sizes and in the launch
configuration the benchmark times, against the FP64 brute force (oracle A) on
seeded ray samples: the microlensing refinement schedule replayed as one HIP
graph (1e6 halo particles + 1e5 point-mass stars, 256^2 base cells, six
rounds), and the 64 batched lenses in one persistent launch."""
import numpy as np
import pytest

import synth
from gpu_helpers import rel_err, say, stats

pytestmark = pytest.mark.gpu

THETA, ORDER, LEAF = 0.3, 8, 16  # the benchmark's settings


def d(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def errors(got, ref):
    """e_alpha, e_kappa, e_gamma per ray; where the brute-force kappa is 0 (a ray
    outside every particle's support) the walk's kappa must be exactly 0 too."""
    ea, ek, eg = rel_err(got, ref)
    zero = ref[:, 2] == 0
    assert np.all(got[zero, 2] == 0.0)
    ek = np.where(zero, 0.0, ek)
    return ea, ek, eg


def test_microlensing_refinement_graph_full_size(ora):
    import paper_1312_1128_amd as g
    import torch

    lens, cx, cy, side = synth.workload_microlensing()
    say(f"[gpu] full-size refinement: n={lens.n}, base {cx.size} cells")
    tree = g.Tree().build(d(lens.x), d(lens.y), d(lens.m), d(lens.s), theta=THETA, q=lens.q, leaf_size=LEAF,
                          order=ORDER)
    run = g.RefinementRun(tree, d(cx), d(cy), d(side), g.refine_schedule(cx.size))
    n = run.run()
    graph = run.capture()
    for v in run.out.values():
        v.zero_()
    graph.replay()
    torch.cuda.synchronize()
    assert n == sum(run.sizes)
    px, py = run.cx[:n].cpu().numpy(), run.cy[:n].cpu().numpy()
    got_all = np.stack([run.out[k][:n].double().cpu().numpy() for k in ["a1", "a2", "kappa", "g1", "g2"]], axis=1)
    a = 0
    for r, size in enumerate(run.sizes):
        idx = a + synth.sample_rays(np.zeros(size), None, 512, 470 + r)
        ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, px[idx], py[idx])
        ea, ek, eg = errors(got_all[idx], ref)
        say(f"  round {r} ({size} rays): max e_alpha {ea.max():.2e} e_kappa {ek.max():.2e} e_gamma {eg.max():.2e}")
        assert ea.max() <= 1e-4 and ek.max() <= 1e-4 and eg.max() <= 1e-4, r
        a += size


def test_batched_64_lenses_full_size(ora):
    """The 64 lenses autotuned as the benchmark does (one order for the batch,
    theta and leaf size per lens, each accepted on 16,384 random rays plus the
    4,096 nearest its densest point), then walked in one persistent launch."""
    import paper_1312_1128_amd as g
    import torch

    lenses = synth.workload_batched_lenses(64)
    say(f"[gpu] full-size batch: {sum(l.n for l, _, _ in lenses)} particles, "
        f"{sum(rx.size for _, rx, _ in lenses)} rays")
    dl = [(d(l.x), d(l.y), d(l.m), d(l.s), d(rx), d(ry)) for l, rx, ry in lenses]
    order, picks, _ = g.autotune_batch(dl, q=lenses[0][0].q)
    assert order is not None
    say(f"  tuned order {order}; (theta, leaf) per lens: {[(p['theta'], p['leaf_size']) for p in picks]}")
    trees = [g.Tree().build(x, y, m, s, theta=p["theta"], q=l.q, leaf_size=p["leaf_size"], order=order)
             for (x, y, m, s, _, _), p, (l, _, _) in zip(dl, picks, lenses)]
    rays = [(d(rx), d(ry)) for _, rx, ry in lenses]
    outs = [{k: torch.empty(r[0].numel(), dtype=torch.float32, device="cuda") for k in ["a1", "a2", "kappa", "g1", "g2"]}
            for r in rays]
    ws = torch.empty(g.batch.batched_workspace_bytes([r[0].numel() for r in rays]), dtype=torch.uint8, device="cuda")
    g.shoot_batched(trees, rays, outs=outs, workspace=ws)
    torch.cuda.synchronize()
    errs = []
    for i, ((l, rx, ry), o) in enumerate(zip(lenses, outs)):
        idx = synth.sample_rays(rx, ry, 128, 500 + i)
        got = np.stack([o[k][idx].double().cpu().numpy() for k in ["a1", "a2", "kappa", "g1", "g2"]], axis=1)
        ref = ora.direct(l.x, l.y, l.m, l.s, l.q, rx[idx], ry[idx])
        errs.append(np.stack(errors(got, ref), axis=1))
    e = np.concatenate(errs)
    stats("e_alpha", e[:, 0])
    stats("e_kappa", e[:, 1])
    stats("e_gamma", e[:, 2])
    assert e[:, 0].max() <= 1e-4 and e[:, 1].max() <= 1e-4 and e[:, 2].max() <= 1e-4
