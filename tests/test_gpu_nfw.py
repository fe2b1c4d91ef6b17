"""Truncated NFW halos as tree particles (Sec. 3.2) on the device, through the
C ABI, against the CPU oracle: the same tree and decisions as the oracle's
tree (topology, big-particle lists and per-ray counts exactly), the FP64 and
FP32 direct sums against the oracle's direct sum, and the paper's halo tests
of Sec. 5.1 (kappa from the halos that hold the ray only, so its error does
not depend on theta; alpha converges as theta falls)."""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_matches_oracle_tree, dev, rel_err, say, shoot, stats

pytestmark = pytest.mark.gpu


def halo_build(lens, c, theta, leaf, order):
    import paper_1312_1128_amd as g

    return g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=theta, q=c, leaf_size=leaf,
                          order=order, nfw=True)


def halos_and_stars(nhalo, nstar, seed):
    """A halo field plus point-mass stars (s = 0) in a small square."""
    lens, c = synth.nfw_halo_field(nhalo, seed)
    stars = synth.star_patch(nstar, seed + 1, center=(0.2, -0.1), side=0.05)
    return synth.Lens(np.concatenate([lens.x, stars.x]), np.concatenate([lens.y, stars.y]),
                      np.concatenate([lens.m, stars.m]), np.concatenate([lens.s, np.zeros(nstar)]), q=c), c


def special_rays(lens, rx, ry):
    """Rays exactly at three halo centres, on a halo's edge, and just inside it."""
    i = np.argsort(-lens.s)[:3]
    ex = np.concatenate([lens.x[i], [lens.x[i[0]] + lens.s[i[0]], lens.x[i[1]] + 0.999999 * lens.s[i[1]]]])
    ey = np.concatenate([lens.y[i], [lens.y[i[0]], lens.y[i[1]]]])
    return np.concatenate([ex, rx]), np.concatenate([ey, ry])


CASES = {
    # (lens, theta, leaf, order)
    "halo_field_3k": (lambda: synth.nfw_halo_field(3000, 301), 0.5, 8, 4),
    "halos_and_stars": (lambda: halos_and_stars(2000, 500, 303), 0.3, 8, 6),
    "halo_field_leaf1": (lambda: synth.nfw_halo_field(1500, 305, rmax=0.05), 0.4, 1, 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_nfw_tree_matches_oracle_tree(ora, case):
    make, theta, leaf, order = CASES[case]
    lens, c = make()
    say(f"[gpu] NFW {case}: n={lens.n} c={c} theta={theta} leaf={leaf} p={order}")
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, theta, leaf, order, nfw=True)
    ex = T.export()
    tree = halo_build(lens, c, theta, leaf, order)
    gx = tree.export()
    assert gx["check_flags"] == 0 and gx["ncells"] == T.ncells
    np.testing.assert_array_equal(gx["next"], ex["next"])
    np.testing.assert_array_equal(gx["lend"] - gx["lbeg"], ex["nl"])
    for cc in np.nonzero(gx["lend"] > gx["lbeg"])[0]:
        np.testing.assert_array_equal(np.sort(gx["list_idx"][gx["lbeg"][cc]:gx["lend"][cc]]), T.list_of(cc))
    assert tree.info()["nlisted"] > 0
    rx, ry = synth.ray_grid(67, -0.9, 0.9)  # 4489 rays: 70 groups and a ragged tail
    rx, ry = special_rays(lens, rx, ry)
    ref, rcnt = T.shoot(rx, ry, counts=True)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    assert rcnt[:, 4].sum() > 0  # some rays fall inside listed halos
    ea, ek, eg = rel_err(got, ref)
    stats("alpha vs oracle tree", ea)
    assert np.quantile(ea, 0.999) < 5e-6 and ea.max() < 2e-5
    ok = ref[:, 2] > 0
    stats("kappa vs oracle tree", ek[ok])
    assert np.all(ek[ok] < 5e-6)
    assert_matches_oracle_tree(got, ref)


def test_nfw_direct_sums(ora):
    import paper_1312_1128_amd as g
    import torch

    lens, c = halos_and_stars(3000, 300, 311)
    rx, ry = synth.uniform_points(2000, 312, -0.9, 0.9)
    rx, ry = special_rays(lens, rx, ry)
    say(f"[gpu] NFW direct sums: n={lens.n} rays={rx.size}")
    ref = ora.direct_nfw(lens.x, lens.y, lens.m, lens.s, c, rx, ry)
    names = ["a1", "a2", "kappa", "g1", "g2"]
    o64 = g.shoot_direct(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), c, dev(rx), dev(ry), fp64=True, nfw=True)
    o32 = g.shoot_direct(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), c, dev(rx), dev(ry), nfw=True)
    torch.cuda.synchronize()
    d64 = np.stack([o64[k].cpu().numpy() for k in names], axis=1)
    d32 = np.stack([o32[k].double().cpu().numpy() for k in names], axis=1)
    # FP64: the same sum term by term, to rounding
    ok = ref[:, 2] > 0
    ea, ek, eg = rel_err(d64, ref)
    stats("FP64 direct alpha", ea)
    assert ea.max() <= 1e-10 and eg.max() <= 1e-10 and np.all(ek[ok] <= 1e-10)
    assert np.all(d64[~ok, 2] == 0.0)
    ea, ek, eg = rel_err(d32, ref)
    stats("FP32 direct alpha", ea)
    assert ea.max() < 1e-5 and np.all(ek[ok] < 1e-5)
    assert np.all(d32[~ok, 2] == 0.0)
    # the tree at theta = 0 is the same direct sum
    tree = halo_build(lens, c, 0.0, 8, 2)
    got = shoot(tree, rx, ry)
    ea, ek, _ = rel_err(got, ref)
    assert ea.max() < 1e-5 and np.all(ek[ok] < 1e-5)


@pytest.mark.parametrize("which", ["E3", "E4"])
def test_nfw_halo_test_kappa_exact_alpha_converges(ora, which):
    """Sec. 5.1: E3 is 10,000 halos of sizes up to 0.3, E4 100 halos of sizes
    up to 0.2, uniform in the unit disk, dN/dm ~ m^-2 on [1e-3, 1], c = 3.
    kappa is exact while an accepted box cannot hide an unlisted halo that
    holds the ray: with lists at support > side / 2 and r_cm the distance to
    the farthest corner (at least side / sqrt 2), that is theta <= 1 / (1 + 1 / sqrt 2)."""
    n, rmax = (10_000, 0.3) if which == "E3" else (100, 0.2)
    lens, c = synth.nfw_halo_field(n, synth.BASE_SEED + 40 + n, rmax=rmax)
    rx, ry = synth.uniform_points(4096, synth.BASE_SEED + 41, -0.9, 0.9)
    ref = ora.direct_nfw(lens.x, lens.y, lens.m, lens.s, c, rx, ry)
    say(f"[gpu] NFW {which}: n={n} rmax={rmax} rays={rx.size}")
    ok = ref[:, 2] > 0
    assert ok.mean() > 0.5
    med = []
    for theta in (0.58, 0.5, 0.3, 0.1):
        got = shoot(halo_build(lens, c, theta, 8, 6), rx, ry)
        ea, ek, _ = rel_err(got, ref)
        say(f"  theta={theta}: alpha median {np.median(ea):.2e} max {ea.max():.2e}; kappa max {ek[ok].max():.2e}")
        # kappa: only halos that hold the ray contribute, at every theta
        assert np.all(ek[ok] < 2e-5) and np.all(got[~ok, 2] == 0.0)
        med.append(np.median(ea))
    assert med[0] > med[1] > med[2] > med[3]
    assert med[3] < 1e-5


def test_nfw_batched_and_rejections():
    import paper_1312_1128_amd as g
    import torch

    lens_a, c = synth.nfw_halo_field(2000, 321)
    lens_b, _ = synth.nfw_halo_field(500, 322, rmax=0.1)
    ta, tb = halo_build(lens_a, c, 0.5, 8, 4), halo_build(lens_b, c, 0.5, 8, 4)
    ra = synth.uniform_points(3000, 323, -0.9, 0.9)
    rb = synth.uniform_points(700, 324, -0.9, 0.9)
    say("[gpu] NFW batched walk vs single walks")
    outs = g.shoot_batched([ta, tb], [(dev(ra[0]), dev(ra[1])), (dev(rb[0]), dev(rb[1]))])
    torch.cuda.synchronize()
    for (tree, (rx, ry)), o in zip([(ta, ra), (tb, rb)], outs):
        single = shoot(tree, rx, ry)
        both = np.stack([o[k].double().cpu().numpy() for k in ["a1", "a2", "kappa", "g1", "g2"]], axis=1)
        ea, ek, _ = rel_err(both, single)
        assert ea.max() < 1e-6
        ok = single[:, 2] > 0
        assert np.all(ek[ok] < 1e-6)
    # a batch mixes no particle kinds
    gauss = synth.nfw_halo(2000, 325)
    tg = g.Tree().build(dev(gauss.x), dev(gauss.y), dev(gauss.m), dev(gauss.s), theta=0.5, q=3.0, leaf_size=8,
                        order=4)
    with pytest.raises(g.GlamerError):
        g.shoot_batched([ta, tg], [(dev(ra[0]), dev(ra[1])), (dev(rb[0]), dev(rb[1]))])



def test_nfw_potential_and_time_delay(ora):
    """psi of a halo field (alpha = grad psi, Sec. 3.2): against the oracle
    tree's psi on the same decisions and the FP64 direct sum; the time delay
    |alpha|^2 / 2 - psi from the same walk."""
    import paper_1312_1128_amd as g
    import torch

    lens, c = halos_and_stars(3000, 400, 341)
    rx, ry = synth.ray_grid(67, -0.9, 0.9)
    rx, ry = special_rays(lens, rx, ry)
    say(f"[gpu] NFW potential: n={lens.n} rays={rx.size}")
    for theta, order in ((0.0, 2), (0.4, 8)):
        tree = halo_build(lens, c, theta, 8, order)
        out = g.shoot_potential(tree, dev(rx), dev(ry))
        torch.cuda.synchronize()
        psi = out["psi"].double().cpu().numpy()
        ref_t = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, theta, 8, order, nfw=True).shoot_psi(rx, ry)
        ref_d = ora.direct_nfw_psi(lens.x, lens.y, lens.m, lens.s, c, rx, ry)
        sc = np.abs(ref_d).max()
        et, ed = np.abs(psi - ref_t).max() / sc, np.abs(psi - ref_d).max() / sc
        say(f"  theta={theta}: psi vs oracle tree {et:.2e}, vs direct {ed:.2e} (of max |psi|)")
        assert et <= 2e-6 and ed <= (2e-6 if theta == 0.0 else 1e-4)
        a = shoot(tree, rx, ry)[:, :2]
        td = out["tdelay"].double().cpu().numpy()
        ref_td = 0.5 * (a[:, 0] ** 2 + a[:, 1] ** 2) - psi
        np.testing.assert_allclose(td, ref_td, rtol=1e-5, atol=1e-6 * np.abs(ref_td).max())


@pytest.mark.parametrize("theta,order", [(0.0, 2), (0.4, 6)])
def test_nfw_adjoint_matches_oracle_tree(ora, theta, order):
    """dL/d(m, x, y, R) of a halo field plus stars for L = sum ga . alpha (+ gk
    kappa + gg . gamma), against the oracle tree's FP64 adjoint on the same
    decisions (at theta = 0: the brute-force gradient)."""
    import paper_1312_1128_amd as g
    import torch

    lens, c = halos_and_stars(2000, 300, 351)
    rx, ry = synth.uniform_points(2500, 352, -0.9, 0.9)
    g0 = synth.rng(353)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    ga, gk, gg = f32(g0.normal(size=(rx.size, 2))), f32(g0.normal(size=rx.size)), f32(g0.normal(size=(rx.size, 2)))
    tree = halo_build(lens, c, theta, 8, order)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, theta, 8, order, nfw=True)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    say(f"[gpu] NFW adjoint theta={theta} p={order}: n={lens.n} rays={rx.size}")
    for with_kg in (False, True):
        kw = dict(gk=t32(gk), gg1=t32(gg[:, 0]), gg2=t32(gg[:, 1])) if with_kg else {}
        got = g.shoot_adjoint(tree, dev(rx), dev(ry), t32(ga[:, 0]), t32(ga[:, 1]), **kw)
        torch.cuda.synchronize()
        ref = T.grad(rx, ry, ga, gk=gk if with_kg else None, gg=gg if with_kg else None)
        for name, a, b in zip(["dL/dm", "dL/dx", "dL/dy", "dL/dR"], got, ref):
            a = a.cpu().numpy()
            sc = np.abs(b).max()
            err = np.abs(a - b)
            say(f"  {'kg ' if with_kg else ''}{name}: max |err|/max|ref| {err.max() / sc:.3e}")
            assert np.all(err <= 1e-4 * np.abs(b) + 2e-6 * sc), name
