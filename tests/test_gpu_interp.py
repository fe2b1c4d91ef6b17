"""Interpolation shortcut of refinement (Sec. 3.4) on the device, against the
oracle's statement of the rule (oracle/refine.py: decisions, neighbours,
shoot lists bit for bit; filled values to FP32 rounding), and against the tree
walk at the interpolated points (the paper finds interpolation and direct
shooting agree to a part in 1e4 for the deflection)."""
import numpy as np
import pytest

import synth
from gpu_helpers import build, dev, say

pytestmark = pytest.mark.gpu

NAMES = ["a1", "a2", "kappa", "g1", "g2"]


def micro_lens(nhalo, nstars, seed):
    halo = synth.nfw_halo(nhalo, seed)
    stars = synth.star_patch(nstars, seed + 2)
    return synth.Lens(np.concatenate([halo.x, stars.x]), np.concatenate([halo.y, stars.y]),
                      np.concatenate([halo.m, stars.m]), np.concatenate([halo.s, stars.s]))


def smooth_lens(nhalo, seed):
    return synth.nfw_halo(nhalo, seed)


# (lens, base cells per side, patch side, patch centre): a smooth halo, where
# the refined cells are mostly uniform, and a star field, where they are not
CASES = {
    "smooth_halo": (lambda: smooth_lens(50_000, 503), 48, 0.0002, (0.3, 0.05)),
    "star_field": (lambda: micro_lens(50_000, 2_000, 501), 48, 0.01, (0.25, 0.0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_interp_rounds_match_rule_and_walk(ora, case):
    import paper_1312_1128_amd as g
    import torch

    make, nbase, patch, (xc, yc) = CASES[case]
    lens = make()
    x0, y0 = xc - patch / 2, yc - patch / 2
    h0 = patch / nbase
    bx, by = synth.ray_grid(nbase, 0.0, patch)
    bx, by = bx + x0, by + y0
    sched = g.refine_schedule(bx.size, rounds=4)
    cap = bx.size + 8 * sum(sched)
    say(f"[gpu] interpolation rounds: n={lens.n} base={nbase}^2 schedule={sched}")
    tree = build(lens, 0.3, 16, 8)
    cx = torch.zeros(cap, dtype=torch.float64, device="cuda")
    cy, side = torch.zeros_like(cx), torch.zeros_like(cx)
    cx[: bx.size], cy[: bx.size], side[: bx.size] = dev(bx), dev(by), h0
    out = {q: torch.zeros(cap, dtype=torch.float32, device="cuda") for q in NAMES}
    n = bx.size
    o0 = g.shoot(tree, cx[:n], cy[:n])
    for q in NAMES:
        out[q][:n] = o0[q]
    lib = g._capi.load()
    import ctypes

    sbytes = ctypes.c_size_t()
    lib.glm_interp_state_bytes(cap, ctypes.byref(sbytes))
    state = torch.empty(sbytes.value, dtype=torch.uint8, device="cuda")
    g.interp_init(cx, cy, n, x0, y0, h0, cap, state)
    idx = torch.zeros(8 * max(sched), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    refined = torch.zeros(max(sched), dtype=torch.int32, device="cuda")
    # the oracle's copy of the grid, fed the device's walked values
    from oracle import refine

    G = refine.NestedGrid(bx, by, x0, y0, h0, nbase, cap)
    for q in NAMES:
        G.out[q][:n] = out[q][:n].cpu().numpy().astype(np.float64)
    interpolated = []
    for r, k in enumerate(sched):
        order, uniform, shoot = G.interp_round(k, 1e-4)
        g.refine_interp_round(cx, cy, side, out, n, k, nbase, 1e-4, cap, state, idx, count, refined=refined)
        cnt = int(count.item())
        say(f"  round {r}: refine {k}, uniform {int(uniform.sum())}, walk {cnt}")
        np.testing.assert_array_equal(refined[:k].cpu().numpy(), order)
        assert cnt == shoot.size
        np.testing.assert_array_equal(idx[:cnt].cpu().numpy(), shoot)
        m = n + 8 * k
        np.testing.assert_array_equal(cx[:m].cpu().numpy(), G.cx[:m])
        np.testing.assert_array_equal(cy[:m].cpu().numpy(), G.cy[:m])
        np.testing.assert_array_equal(side[:m].cpu().numpy(), G.side[:m])
        filled = np.setdiff1d(np.arange(n, m), shoot)
        for q in NAMES:
            if filled.size == 0:
                break
            got = out[q][:m].cpu().numpy()[filled].astype(np.float64)
            np.testing.assert_allclose(got, G.out[q][filled], rtol=1e-6, atol=1e-7 * np.abs(G.out[q][filled]).max())
        g.shoot_indexed(tree, cx, cy, idx, cnt, out)
        for q in NAMES:  # the device values (walked, and filled up to rounding) carry over to the oracle's grid
            G.out[q][n:m] = out[q][n:m].cpu().numpy().astype(np.float64)
        interpolated.append(filled)
        n = m
    interpolated = np.concatenate(interpolated)
    say(f"  {interpolated.size} of {n - bx.size} new cells interpolated")
    if case == "smooth_halo":
        assert interpolated.size > (n - bx.size) // 2
    if interpolated.size == 0:
        return
    # interpolated cells against walking the same points
    walked = g.shoot(tree, dev(G.cx[interpolated]), dev(G.cy[interpolated]))
    a_int = np.stack([out["a1"].cpu().numpy()[interpolated], out["a2"].cpu().numpy()[interpolated]], 1)
    a_w = np.stack([walked["a1"].cpu().numpy(), walked["a2"].cpu().numpy()], 1).astype(np.float64)
    err = np.linalg.norm(a_int - a_w, axis=1) / np.linalg.norm(a_w, axis=1)
    say(f"  {interpolated.size} interpolated rays: alpha vs walk max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() <= 1e-4
    dk = np.abs(out["kappa"].cpu().numpy()[interpolated] - walked["kappa"].cpu().numpy())
    say(f"  kappa vs walk max {dk.max():.2e}")
    # and against the FP64 brute force at a sample of the interpolated points
    pick = interpolated[synth.sample_rays(interpolated, None, 256, 509)]
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, G.cx[pick], G.cy[pick])
    a_i = np.stack([out["a1"].cpu().numpy()[pick], out["a2"].cpu().numpy()[pick]], 1).astype(np.float64)
    eb = np.linalg.norm(a_i - ref[:, :2], axis=1) / np.linalg.norm(ref[:, :2], axis=1)
    say(f"  interpolated alpha vs brute force ({pick.size} rays): max {eb.max():.2e}")
    assert eb.max() <= 1e-4


def test_interp_tol_zero_walks_everything():
    import paper_1312_1128_amd as g
    import torch

    lens = micro_lens(20_000, 500, 511)
    nbase, patch = 32, 0.01
    x0, y0 = 0.25 - patch / 2, -patch / 2
    bx, by = synth.ray_grid(nbase, 0.0, patch)
    tree = build(lens, 0.3, 16, 8)
    sched = g.refine_schedule(bx.size, rounds=3)
    run = g.RefinementRun(tree, dev(bx + x0), dev(by + y0), dev(np.full(bx.size, patch / nbase)), sched)
    n = run.run()
    torch.cuda.synchronize()
    plain = {q: v[:n].cpu().numpy().copy() for q, v in run.out.items()}
    pos = (run.cx[:n].cpu().numpy().copy(), run.cy[:n].cpu().numpy().copy(), run.side[:n].cpu().numpy().copy())
    n2, walked = run.run_interp(x0, y0, patch / nbase, nbase, tol=0.0)
    torch.cuda.synchronize()
    say(f"[gpu] tol 0: {n2} cells, {walked} walked")
    assert n2 == n
    np.testing.assert_array_equal(run.cx[:n].cpu().numpy(), pos[0])
    np.testing.assert_array_equal(run.side[:n].cpu().numpy(), pos[2])
    # with tol 0 only exactly equal neighbourhoods are interpolated
    for q in NAMES:
        np.testing.assert_allclose(run.out[q][:n].cpu().numpy(), plain[q], rtol=2e-5,
                                   atol=1e-6 * np.abs(plain[q]).max())


def test_interp_invalid_arguments():
    import paper_1312_1128_amd as g
    import torch

    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    st = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GlamerError):  # state too small
        g.interp_init(x, x, 16, 0.0, 0.0, 1.0, 16, st)
    with pytest.raises(g.GlamerError):  # bad base grid
        g.interp_init(x, x, 16, 0.0, 0.0, 0.0, 16, torch.empty(1 << 16, dtype=torch.uint8, device="cuda"))


# ------------------------------------------------------------ deflection mode

def test_interp_deflection_mode_matches_rule(ora):
    """Refinement with deflection-only walks: the base cells and each round's
    walked cells get kappa, gamma from the three-point magnification matrix
    (App. A), and the uniformity test compares the pair estimates of A; all
    against the oracle's statement of the rule (decisions and walk lists bit
    for bit, values to FP32 rounding)."""
    from oracle import refine

    import paper_1312_1128_amd as g
    import torch

    # five large truncated NFW halos: a deflection field smooth on the cell scale,
    # where FP32 deflections still resolve A to ~1e-4
    lens, c = synth.nfw_halo_field(5, 9, rmax=1.5)
    nbase, patch, (xc, yc), tol = 32, 0.02, (0.3, 0.05), 1e-3
    x0, y0 = xc - patch / 2, yc - patch / 2
    h0 = patch / nbase
    bx, by = synth.ray_grid(nbase, 0.0, patch)
    bx, by = bx + x0, by + y0
    sched = g.refine_schedule(bx.size, rounds=3)
    cap = bx.size + 8 * sum(sched)
    say(f"[gpu] interpolation, deflection mode: n={lens.n} halos, base={nbase}^2 schedule={sched}")
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=0.3, q=c, leaf_size=16, order=8,
                          nfw=True)
    cx = torch.zeros(cap, dtype=torch.float64, device="cuda")
    cy, side = torch.zeros_like(cx), torch.zeros_like(cx)
    n = bx.size
    cx[:n], cy[:n], side[:n] = dev(bx), dev(by), h0
    out = {q: torch.zeros(cap, dtype=torch.float32, device="cuda") for q in NAMES}
    lib = g._capi.load()
    import ctypes

    sbytes = ctypes.c_size_t()
    lib.glm_interp_state_bytes(cap, ctypes.byref(sbytes))
    state = torch.empty(sbytes.value, dtype=torch.uint8, device="cuda")
    g.interp_init(cx, cy, n, x0, y0, h0, cap, state)
    g.shoot_indexed(tree, cx, cy, torch.arange(n, dtype=torch.int32, device="cuda"), n, out, alpha_only=True)
    g.interp_estimate(cx, cy, out, nbase, cap, state, max_count=n)
    G = refine.NestedGrid(bx, by, x0, y0, h0, nbase, cap)
    for q in NAMES:
        G.out[q][:n] = out[q][:n].cpu().numpy().astype(np.float64)
    est = G.estimate_kg(range(n)).astype(np.float32).astype(np.float64)
    got = np.stack([G.out["kappa"][:n], G.out["g1"][:n], G.out["g2"][:n]], axis=1)
    np.testing.assert_allclose(got, est, rtol=1e-6, atol=1e-6 * np.abs(est).max())
    idx = torch.zeros(8 * max(sched), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    refined = torch.zeros(max(sched), dtype=torch.int32, device="cuda")
    filled_all = []
    for r, k in enumerate(sched):
        order, uniform, shoot = G.interp_round(k, tol, deflections=True)
        g.refine_interp_round(cx, cy, side, out, n, k, nbase, tol, cap, state, idx, count, refined=refined,
                              deflections=True)
        cnt = int(count.item())
        say(f"  round {r}: refine {k}, uniform {int(uniform.sum())}, walk {cnt}")
        np.testing.assert_array_equal(refined[:k].cpu().numpy(), order)
        assert cnt == shoot.size
        np.testing.assert_array_equal(idx[:cnt].cpu().numpy(), shoot)
        m = n + 8 * k
        np.testing.assert_array_equal(cx[:m].cpu().numpy(), G.cx[:m])
        filled = np.setdiff1d(np.arange(n, m), shoot)
        for q in NAMES:
            if filled.size:
                gq = out[q][:m].cpu().numpy()[filled].astype(np.float64)
                np.testing.assert_allclose(gq, G.out[q][filled], rtol=1e-6,
                                           atol=1e-7 * np.abs(G.out[q][filled]).max())
        g.shoot_indexed(tree, cx, cy, idx, cnt, out, alpha_only=True)
        g.interp_estimate(cx, cy, out, nbase, cap, state, idx=idx, count=count, max_count=8 * k)
        for q in ("a1", "a2"):
            G.out[q][shoot] = out[q].cpu().numpy()[shoot].astype(np.float64)
            G.out[q][filled] = out[q].cpu().numpy()[filled].astype(np.float64)
        est = G.estimate_kg(shoot).astype(np.float32).astype(np.float64)
        got = np.stack([out[q].cpu().numpy()[shoot].astype(np.float64) for q in ("kappa", "g1", "g2")], axis=1)
        np.testing.assert_allclose(got, est, rtol=1e-6, atol=1e-6 * max(np.abs(est).max(), 1e-30))
        for q in ("kappa", "g1", "g2"):
            G.out[q][n:m] = out[q].cpu().numpy()[n:m].astype(np.float64)
        filled_all.append(filled)
        n = m
    filled_all = np.concatenate(filled_all)
    say(f"  {filled_all.size} of {n - bx.size} new cells interpolated")
    assert filled_all.size > 0
    walked = g.shoot(tree, dev(G.cx[filled_all]), dev(G.cy[filled_all]), alpha_only=True)
    a_int = np.stack([out["a1"].cpu().numpy()[filled_all], out["a2"].cpu().numpy()[filled_all]], 1)
    a_w = np.stack([walked["a1"].cpu().numpy(), walked["a2"].cpu().numpy()], 1).astype(np.float64)
    err = np.linalg.norm(a_int - a_w, axis=1) / np.linalg.norm(a_w, axis=1)
    say(f"  interpolated alpha vs walk: max {err.max():.2e} median {np.median(err):.2e}")
    assert err.max() <= 1e-3
    pick = filled_all[synth.sample_rays(filled_all, None, 256, 519)]
    ref = ora.direct_nfw(lens.x, lens.y, lens.m, lens.s, c, G.cx[pick], G.cy[pick])
    a_i = np.stack([out["a1"].cpu().numpy()[pick], out["a2"].cpu().numpy()[pick]], 1).astype(np.float64)
    eb = np.linalg.norm(a_i - ref[:, :2], axis=1) / np.linalg.norm(ref[:, :2], axis=1)
    say(f"  interpolated alpha vs brute force ({pick.size} rays): max {eb.max():.2e}")
    assert eb.max() <= 1e-3
