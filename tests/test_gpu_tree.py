"""GPU parity of the tree build and the forward walk (through the C ABI)
against the CPU oracle: oracle B (same tree definition) must agree on the
topology exactly and on the per-ray interaction counts exactly; oracle A (brute
force) bounds the approximation of the whole method."""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_matches_oracle_tree, build, dev, rel_err, say, shoot, stats

pytestmark = pytest.mark.gpu


def mixed_lens(n, seed, s_lo=0.003, s_hi=0.3, frac_points=0.2):
    lens = synth.gaussian_blobs(n, seed, s_lo=s_lo, s_hi=s_hi)
    g = synth.rng(seed + 1)
    lens.s[g.random(n) < frac_points] = 0.0
    return lens


CASES = {
    "point_masses_1k": (lambda: synth.point_masses(1000, synth.BASE_SEED + 1), 0.5, 8, 2),
    "nfw_20k": (lambda: synth.nfw_halo(20000, synth.BASE_SEED + 3), 0.3, 8, 6),
    "mixed_3k_leaf3": (lambda: mixed_lens(3000, 17), 0.5, 3, 4),
    "mixed_5k_leaf1": (lambda: mixed_lens(5000, 19), 0.4, 1, 3),
}


def compare_topology(ora, lens, theta, leaf, order, tree=None):
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, leaf, order)
    ex = T.export()
    if tree is None:
        tree = build(lens, theta, leaf, order)
    else:  # rebuild the given handle
        tree.build(dev(lens.x), dev(lens.y), dev(lens.m), dev(lens.s), theta=theta, q=lens.q, leaf_size=leaf,
                   order=order)
    g = tree.export()
    assert g["check_flags"] == 0
    nc = T.ncells
    assert g["ncells"] == nc, (g["ncells"], nc)
    np.testing.assert_array_equal(g["level"], ex["level"])
    np.testing.assert_array_equal(g["ix"], ex["ix"])
    np.testing.assert_array_equal(g["iy"], ex["iy"])
    np.testing.assert_array_equal(g["end"] - g["beg"], ex["np"])
    np.testing.assert_array_equal(g["leaf"], ex["leaf"])
    np.testing.assert_array_equal(g["next"], ex["next"])
    np.testing.assert_array_equal(g["lend"] - g["lbeg"], ex["nl"])
    x0, y0, S = T.root()
    assert (g["root_x0"], g["root_y0"], g["root_side"]) == (x0, y0, S)
    # every leaf holds the same particles; every list the same particles
    perm = g["perm"]
    for c in np.nonzero(g["leaf"])[0]:
        np.testing.assert_array_equal(np.sort(perm[g["beg"][c]:g["end"][c]]), T.members(c))
    for c in np.nonzero(g["lend"] > g["lbeg"])[0]:
        np.testing.assert_array_equal(np.sort(g["list_idx"][g["lbeg"][c]:g["lend"][c]]), T.list_of(c))
    # moments (FP64, bottom-up on the GPU vs directly from the members)
    np.testing.assert_allclose(g["M"], ex["M"], rtol=1e-12)
    side = S / 2.0 ** ex["level"]
    assert np.all(np.abs(g["cx"] - ex["cx"]) <= 1e-12 * np.maximum(side, 1e-300) + 1e-15)
    assert np.all(np.abs(g["cy"] - ex["cy"]) <= 1e-12 * np.maximum(side, 1e-300) + 1e-15)
    # r_cut = r_cm / theta moves with the centre of mass: by at most what the
    # tolerance above allows for it (the bound that decides at boxes ~1e-7 across)
    dr = np.sqrt(2.0) * (1e-12 * np.maximum(side, 1e-300) + 1e-15) / theta
    assert np.all(np.abs(g["rcut2"] - ex["rcut2"]) <= 1e-10 * ex["rcut2"] + 2 * np.sqrt(ex["rcut2"]) * dr + dr * dr)
    # Q_k about the centre of mass: a shift dz of the centre moves it by
    # k dz Q_{k-1}, |Q_{k-1}| <= M (sqrt(2) side)^(k-1); dz as allowed above
    dz = np.sqrt(2.0) * (1e-12 * np.maximum(side, 1e-300) + 1e-15)
    for k in range(order + 1):
        scale = ex["M"] * (np.sqrt(2) * side) ** k
        shift = k * ex["M"] * dz * (np.sqrt(2) * side) ** max(k - 1, 0)
        assert np.all(np.abs(g["Q"][:, k] - ex["Q"][:, k]) <= 1e-10 * scale + shift + 1e-300), k
    return T, tree


@pytest.mark.parametrize("case", list(CASES))
def test_tree_and_walk_match_oracle_tree(ora, case):
    make, theta, leaf, order = CASES[case]
    lens = make()
    say(f"[gpu] {case}: n={lens.n} theta={theta} leaf={leaf} p={order}")
    T, tree = compare_topology(ora, lens, theta, leaf, order)
    rx, ry = synth.ray_grid(67)  # 4489 rays: 70 groups + a ragged tail
    ref, rcnt = T.shoot(rx, ry, counts=True)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    # identical decisions: boxes visited, accepted, leaf particles, list hits
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    ea, ek, eg = rel_err(got, ref)
    stats("alpha vs oracle tree", ea)
    stats("gamma vs oracle tree", eg)
    # measured worst: alpha 5.4e-6 per ray (p99.9 1.3e-6), kappa 1.1e-6
    assert np.quantile(ea, 0.999) < 5e-6 and ea.max() < 2e-5
    if lens.s.max() > 0:
        ok = np.abs(ref[:, 2]) > 0
        stats("kappa vs oracle tree", ek[ok])
        assert np.all(ek[ok] < 5e-6)
    assert_matches_oracle_tree(got, ref)


def test_particle_order_on_every_sort_path(ora):
    """The particles end in the full Morton-key order (equal keys in input
    order) whichever way the build sorted them: on the keys' top 32 bits with
    the runs equal in them ordered afterwards (no box below level 16), on all
    64 bits after finding such a box, and on all 64 bits first when the handle's
    last build had one; each time with the oracle tree's topology."""
    g0 = synth.rng(341)
    base = mixed_lens(4000, 343)
    S = 1.0  # the lenses span about one unit

    def with_clusters(sizes, spread):
        lens = synth.Lens(base.x.copy(), base.y.copy(), base.m.copy(), base.s.copy(), q=base.q)
        at = 0
        for k in sizes:  # k particles within spread * S of particle `at`
            lens.x[at + 1:at + k] = lens.x[at] + spread * S * g0.uniform(-1, 1, k - 1)
            lens.y[at + 1:at + k] = lens.y[at] + spread * S * g0.uniform(-1, 1, k - 1)
            at += k
        return lens

    shallow = with_clusters([2, 3, 5, 2, 4, 3, 6, 2] * 3, 1e-7)  # runs equal in the top bits, none above L
    deep = with_clusters([40, 3, 2], 1e-7)                        # a box below level 16
    deep.x[100:120], deep.y[100:120] = deep.x[100], deep.y[100]   # and 20 coincident ones (the depth cap)
    tree = None
    for name, lens in [("shallow", shallow), ("deep", deep), ("deep again", deep), ("shallow after deep", shallow),
                       ("shallow again", shallow)]:
        say(f"[gpu] sort path: {name}")
        T, tree = compare_topology(ora, lens, 0.5, 8, 3, tree=tree)
        ex = tree.export()
        key, perm = ex["key"], ex["perm"]
        assert np.all(key[1:] >= key[:-1]), name
        eq = key[1:] == key[:-1]
        assert np.all(perm[1:][eq] > perm[:-1][eq]), name
        np.testing.assert_array_equal(np.sort(perm), np.arange(lens.n))
    assert int(eq.sum()) == 0  # the shallow lens has no equal keys, only keys equal in their top bits


def test_massless_boxes_match_oracle_tree(ora):
    """Every particle in one quadrant of the image massless, so that whole boxes
    have M = 0 and take their geometric centre as expansion centre (the rule
    both sides follow); topology, moments, counts and values as above."""
    lens = mixed_lens(4000, 23)
    lens.m[(lens.x < np.median(lens.x)) & (lens.y < np.median(lens.y))] = 0.0
    say(f"[gpu] massless quadrant: n={lens.n}, {int((lens.m == 0).sum())} massless")
    T, tree = compare_topology(ora, lens, 0.5, 4, 6)
    assert (T.export()["M"] == 0).sum() > 10
    rx, ry = synth.ray_grid(50)
    ref, rcnt = T.shoot(rx, ry, counts=True)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    assert_matches_oracle_tree(got, ref)


def test_theta_zero_walk_is_direct_sum(ora):
    lens = mixed_lens(4000, 23)
    say("[gpu] theta=0 walk vs oracle A")
    tree = build(lens, 0.0, 8, 2)
    rx, ry = synth.uniform_points(1000, 24)
    got, cnt = shoot(tree, rx, ry, counts=True)
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx, ry)
    assert np.all(cnt[:, 1] == 0) and np.all(cnt[:, 2] == lens.n)
    ea, ek, eg = rel_err(got, ref)
    stats("alpha", ea)
    stats("gamma", eg)
    assert ea.max() < 1e-5 and ek.max() < 1e-5


def test_headline_nfw_1e6_vs_bruteforce(ora):
    """1e6 smoothed NFW particles (c = 5, kNN32, q = 3), the full 2048^2 ray grid
    shot at theta = 0.3 with p = 8 and leaf size 16 (the benchmark's
    configuration).  16,384 seeded rays plus the 4,096 rays nearest the halo
    centre (where the shear is smallest and its relative error largest) are
    checked against the FP64 brute force: max fractional error <= 1e-4 for
    alpha, kappa and gamma."""
    lens, rx, ry = synth.workload_nfw()
    say(f"[gpu] headline nfw n={lens.n} rays={rx.size}")
    tree = build(lens, 0.3, 16, 8)
    assert tree.info()["check_flags"] == 0
    got, cnt = shoot(tree, rx, ry, counts=True)
    central = np.argsort(rx * rx + ry * ry, kind="stable")[:4096]
    idx = np.union1d(synth.sample_rays(rx, ry, 16384, synth.BASE_SEED + 7), central)
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, rx[idx], ry[idx])
    ea, ek, eg = rel_err(got[idx], ref)
    stats("alpha vs brute force", ea)
    stats("kappa vs brute force", ek)
    stats("gamma vs brute force", eg)
    say(f"  mean counts per ray (visited, accepted, leaf, list hits): {cnt.mean(0)}")
    assert ea.max() <= 1e-4 and ek.max() <= 1e-4 and eg.max() <= 1e-4
    assert np.all(got[idx][ref[:, 2] == 0, 2] == 0.0)
    # the same sampled rays through the oracle tree: identical decisions
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.3, 16, 8)
    refB, rc = T.shoot(rx[idx], ry[idx], counts=True)
    np.testing.assert_array_equal(cnt[idx], rc[:, [0, 1, 2, 4]])


def test_edge_cases(ora):
    import paper_1312_1128_amd as g
    import torch

    say("[gpu] edge cases")
    # one particle; fewer than a leaf; coincident particles (depth cap)
    for n, L in [(1, 8), (5, 8), (9, 8)]:
        lens = mixed_lens(n, 31 + n)
        tree = build(lens, 0.5, L, 4)
        rx, ry = synth.uniform_points(130, 32)
        got = shoot(tree, rx, ry)
        ref = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.5, L, 4).shoot(rx, ry)
        np.testing.assert_allclose(got, ref, rtol=2e-5, atol=1e-6 * np.abs(ref).max())
    lens = synth.point_masses(40, 33)
    lens.x[:20] = 0.1
    lens.y[:20] = -0.2
    tree = build(lens, 0.5, 4, 3)
    inf = tree.info()
    assert inf["max_level"] == 32 and inf["check_flags"] == 0
    rx, ry = synth.uniform_points(64, 34)
    got = shoot(tree, rx, ry)
    ref = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.5, 4, 3).shoot(rx, ry)
    np.testing.assert_allclose(got[:, :2], ref[:, :2], rtol=2e-5, atol=1e-6 * np.abs(ref[:, :2]).max())
    # zero rays and a single ray
    out = g.shoot(tree, dev(np.zeros(0)), dev(np.zeros(0)))
    assert out["a1"].numel() == 0
    got1 = shoot(tree, rx[:1], ry[:1])
    np.testing.assert_allclose(got1[0, :2], ref[0, :2], rtol=2e-5)
    # rays far outside the particles: pure multipoles of the root
    far = shoot(tree, np.array([50.0, -80.0]), np.array([3.0, 40.0]))
    reff = ora.direct(lens.x, lens.y, lens.m, lens.s, 3.0, np.array([50.0, -80.0]), np.array([3.0, 40.0]))
    np.testing.assert_allclose(far[:, :2], reff[:, :2], rtol=1e-5)
    torch.cuda.synchronize()


@pytest.mark.parametrize("leaf,order", [(64, 12), (8, 0), (2, 1)])
def test_parameter_extremes(ora, leaf, order):
    """Largest leaf and order, the monopole alone, and near-singleton leaves."""
    lens = mixed_lens(6000, 27)
    say(f"[gpu] parameter extremes: leaf={leaf} p={order}")
    T, tree = compare_topology(ora, lens, 0.45, leaf, order)
    rx, ry = synth.ray_grid(45)
    ref, rcnt = T.shoot(rx, ry, counts=True)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    ea, ek, eg = rel_err(got, ref)
    stats("alpha vs oracle tree", ea)
    assert np.quantile(ea, 0.999) < 5e-6 and ea.max() < 2e-5
    assert_matches_oracle_tree(got, ref)


def test_point_masses_without_smoothing_array(ora):
    """s = NULL: every particle is a point mass; kappa is exactly zero."""
    import paper_1312_1128_amd as g

    lens = synth.point_masses(3000, 29)
    say("[gpu] point masses, s = NULL")
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=0.5, q=3.0, leaf_size=8, order=4)
    assert tree.info()["nlisted"] == 0
    rx, ry = synth.ray_grid(40)
    got, gcnt = shoot(tree, rx, ry, counts=True)
    T = ora.Tree(lens.x, lens.y, lens.m, np.zeros(lens.n), 3.0, 0.5, 8, 4)
    ref, rcnt = T.shoot(rx, ry, counts=True)
    np.testing.assert_array_equal(gcnt, rcnt[:, [0, 1, 2, 4]])
    assert np.all(got[:, 2] == 0.0)
    ea, _, eg = rel_err(got, ref)
    assert ea.max() < 1e-5 and eg.max() < 1e-4


def test_determinism_and_flags(ora):
    import paper_1312_1128_amd as g

    say("[gpu] determinism and flags")
    lens = synth.nfw_halo(30000, 41)
    rx, ry = synth.ray_grid(100)
    tree = build(lens, 0.3, 8, 6)
    a = shoot(tree, rx, ry)
    b = shoot(tree, rx, ry)
    np.testing.assert_array_equal(a, b)  # no atomics in the forward: bitwise repeatable
    tree2 = build(lens, 0.3, 8, 6)
    np.testing.assert_array_equal(shoot(tree2, rx, ry), a)  # rebuild is deterministic too
    ao = shoot(tree, rx, ry, alpha_only=True)
    np.testing.assert_array_equal(ao[:, :2], a[:, :2])
    # rays passed as they are (no ray sort): other groups, same per-ray decisions and arithmetic
    od = shoot(tree, rx, ry, ordered=True)
    np.testing.assert_array_equal(od, a)
    nk = shoot(tree, rx, ry, fp32_alpha=True)  # plain FP32 summation of alpha: ~sqrt(terms) eps
    ea = np.linalg.norm(nk[:, :2] - a[:, :2], axis=1) / np.linalg.norm(a[:, :2], axis=1)
    assert ea.max() < 1e-5


def test_split_walk_matches_single_range(ora):
    """Few rays: the walk splits the box array over several wavefronts per ray
    group; same decisions and counts as the oracle tree, sums regrouped only."""
    lens = synth.nfw_halo(30000, 45)
    rx, ry = synth.uniform_points(700, 46)
    say("[gpu] split walk (700 rays)")
    tree = build(lens, 0.3, 8, 6)
    got, cnt = shoot(tree, rx, ry, counts=True)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.3, 8, 6)
    ref, rc = T.shoot(rx, ry, counts=True)
    np.testing.assert_array_equal(cnt, rc[:, [0, 1, 2, 4]])
    ea, ek, eg = rel_err(got, ref)
    assert ea.max() < 1e-5 and ek.max() < 1e-5
    # the split walk inside one big launch gives the same values per ray
    big_x = np.concatenate([rx, synth.uniform_points(2_000_000, 47)[0]])
    big_y = np.concatenate([ry, synth.uniform_points(2_000_000, 47)[1]])
    got_big = shoot(tree, big_x, big_y)[: rx.size]
    np.testing.assert_allclose(got_big[:, :2], got[:, :2], rtol=2e-6, atol=1e-7 * np.abs(got[:, :2]).max())


def test_split_walk_with_an_empty_last_range(ora):
    """Rays over the whole lens: the box that holds them all is the root, so the
    split walk's last range (the boxes after that box's subtree) is empty.  Its
    wavefronts replay no ancestors: the replay for a range starting at the end
    of the box array used to step past the root's last child (two children
    here, a collinear lens) and read a header beyond the array.  Forward and
    adjoint against the oracle tree."""
    import paper_1312_1128_amd as g
    import torch

    gen = synth.rng(119)
    n = 2000
    t = gen.uniform(0.05, 0.5, n) * np.where(gen.random(n) < 0.5, -1.0, 1.0)
    x, y = t, 0.3 * t * (1.0 + 1e-2 * gen.normal(size=n))  # two opposite quadrants of the root, none near its centre
    s = gen.uniform(0.002, 0.1, n)
    s[gen.random(n) < 0.2] = 0.0
    lens = synth.Lens(x, y, gen.uniform(0.1, 1.0, n) / n, s, q=3.0)
    rx, ry = gen.uniform(-0.6, 0.6, 300), gen.uniform(-0.6, 0.6, 300)
    say("[gpu] split walk with an empty last range (collinear lens, 300 rays)")
    tree = build(lens, 0.4, 4, 5)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.4, 4, 5)
    ex = T.export()
    kids, ch = 0, 1
    while ch < T.ncells:
        kids += 1
        ch = int(ex["next"][ch])
    assert kids <= 2 and T.ncells >= 256  # the case above: a split walk over a root with two children
    got, cnt = shoot(tree, rx, ry, counts=True)
    ref, rc = T.shoot(rx, ry, counts=True)
    np.testing.assert_array_equal(cnt, rc[:, [0, 1, 2, 4]])
    assert_matches_oracle_tree(got, ref)
    ga = synth.rng(121).normal(size=(rx.size, 2)).astype(np.float32).astype(np.float64)
    tt = torch.from_numpy(np.ascontiguousarray(ga, dtype=np.float32)).cuda()
    grads = g.shoot_adjoint(tree, dev(rx), dev(ry), tt[:, 0].contiguous(), tt[:, 1].contiguous())
    torch.cuda.synchronize()
    for name, a, b in zip("mxys", grads, T.grad(rx, ry, ga)):
        a = a.cpu().numpy()
        assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 2e-6 * np.abs(b).max()), name


def test_bad_inputs_are_rejected():
    import paper_1312_1128_amd as g

    say("[gpu] error paths")
    lens = synth.point_masses(100, 51)
    x = lens.x.copy()
    x[7] = np.nan
    with pytest.raises(g.GlamerError) as e:
        g.Tree().build(dev(x), dev(lens.y), dev(lens.m), None)
    assert e.value.status == -5
    m = lens.m.copy()
    m[3] = -1.0
    with pytest.raises(g.GlamerError):
        g.Tree().build(dev(lens.x), dev(lens.y), dev(m), None)
    with pytest.raises(g.GlamerError) as e:
        g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=1.0)
    assert e.value.status == -1
    with pytest.raises(g.GlamerError):
        g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), None, order=13)
    t = g.Tree()
    with pytest.raises(g.GlamerError) as e:
        g.shoot(t, dev(np.zeros(3)), dev(np.zeros(3)))
    assert e.value.status == -4


def test_caller_workspace_contract(ora):
    """The tree lives in the caller's workspace: the bound of
    glm_tree_workspace_bytes holds on a worst case of depth-capped clusters; a
    workspace too small for the boxes is refused after the box count is known
    (with the exact size reported); a build into exactly that size equals one
    into the bound; two trees in two workspaces do not disturb each other."""
    import paper_1312_1128_amd as g
    import torch

    say("[gpu] caller workspace contract")
    # clusters of L + 1 coincident particles: each one a chain of boxes down to the depth cap
    L = 4
    gen = synth.rng(61)
    centres = gen.uniform(-0.5, 0.5, (200, 2))
    pos = np.repeat(centres, L + 1, axis=0)
    lens = synth.Lens(pos[:, 0].copy(), pos[:, 1].copy(), np.full(pos.shape[0], 1e-3), np.zeros(pos.shape[0]))
    p = g.GlmParams(0.5, 3.0, L, 4, 0)
    bound = g.tree_workspace_bytes(lens.n, p)
    tree = g.Tree().build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=0.5, leaf_size=L, order=4)
    need = tree.required_bytes()
    inf = tree.info()
    say(f"  {lens.n} particles: {inf['ncells']} boxes, need {need} of the bound {bound} bytes")
    assert inf["check_flags"] == 0 and inf["max_level"] == 32 and need <= bound and inf["device_bytes"] == need
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, 3.0, 0.5, L, 4)
    assert inf["ncells"] == T.ncells
    rx, ry = synth.uniform_points(500, 62)
    ref = shoot(tree, rx, ry)
    # too small for the boxes: refused after the count, exact need reported
    small = torch.empty(need - 4096, dtype=torch.uint8, device="cuda")
    t2 = g.Tree()
    with pytest.raises(g.GlamerError) as e:
        t2.build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=0.5, leaf_size=L, order=4, workspace=small)
    assert e.value.status == -2
    assert t2.required_bytes() == need
    with pytest.raises(g.GlamerError) as e:
        g.shoot(t2, dev(rx), dev(ry))
    assert e.value.status == -4
    exact = torch.empty(need, dtype=torch.uint8, device="cuda")
    t2.build(dev(lens.x), dev(lens.y), dev(lens.m), None, theta=0.5, leaf_size=L, order=4, workspace=exact)
    np.testing.assert_array_equal(shoot(t2, rx, ry), ref)
    # a second tree in its own workspace; rebuilding it leaves the first intact
    other = synth.nfw_halo(5000, 63)
    t3 = build(other, 0.3, 8, 6)
    a3 = shoot(t3, rx, ry)
    t3.build(dev(other.x[::-1].copy()), dev(other.y[::-1].copy()), dev(other.m), dev(other.s[::-1].copy()),
             theta=0.3, q=other.q, leaf_size=8, order=6)
    np.testing.assert_array_equal(shoot(t2, rx, ry), ref)
    np.testing.assert_array_equal(shoot(tree, rx, ry), ref)
    np.testing.assert_allclose(shoot(t3, rx, ry), a3, rtol=1e-6, atol=1e-7 * np.abs(a3).max())


def test_wavefront_counts_and_list_search(ora):
    """The four wavefront counts (list entries tested, boxes accepted, leaf
    particles and list candidates evaluated) are shared by the 64 rays of a
    group and bound the per-ray counts: every list hit was a tested entry and
    an evaluated candidate, every accepted box and leaf particle of a ray was
    evaluated by its wavefront.  On the 1e6-particle halo the lists whose
    support bounds miss the group are skipped whole, so far fewer entries are
    tested than a per-ray scan of every visited box's list (oracle B's count)."""
    lens, gx, gy = synth.workload_nfw()
    say("[gpu] wavefront counts and list search")
    tree = build(lens, 0.3, 16, 8)
    # a 256 x 256 block of the grid near the centre, listed in 8 x 8 tiles (one group per tile)
    n = 2048
    i0 = n // 2 - 128
    ti, tj = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    ii, jj = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
    gi = (i0 + 8 * ti.reshape(-1, 1) + ii.reshape(1, -1)).ravel()
    gj = (i0 + 8 * tj.reshape(-1, 1) + jj.reshape(1, -1)).ravel()
    rx = -0.5 + (gi + 0.5) / n
    ry = -0.5 + (gj + 0.5) / n
    _, c = shoot(tree, rx, ry, all_counts=True, ordered=True)
    grp = c.reshape(-1, 64, 8)
    for k in range(4, 8):
        assert np.all(grp[:, :, k] == grp[:, :1, k]), k  # one value per group
    assert np.all(c[:, 4] >= c[:, 3]) and np.all(c[:, 7] >= grp[:, :, 3].max(1).repeat(64))
    assert np.all(c[:, 5] >= grp[:, :, 1].max(1).repeat(64))
    assert np.all(c[:, 6] >= grp[:, :, 2].max(1).repeat(64))
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.3, 16, 8)
    _, rc = T.shoot(rx, ry, counts=True)
    np.testing.assert_array_equal(c[:, :4], rc[:, [0, 1, 2, 4]])
    lane_use = [c[:, 1].sum() / (64 * grp[:, 0, 5].sum()), c[:, 2].sum() / (64 * grp[:, 0, 6].sum()),
                c[:, 3].sum() / (64 * grp[:, 0, 7].sum())]
    say(f"  per ray: list entries tested {c[:, 4].mean():.0f} (a per-ray scan of every visited list: "
        f"{rc[:, 3].mean():.0f}), hits {c[:, 3].mean():.0f}; lane use accepted {lane_use[0]:.2f} leaf "
        f"{lane_use[1]:.2f} list {lane_use[2]:.2f}")
    assert c[:, 4].mean() < 0.5 * rc[:, 3].mean()
    assert all(0.3 < u <= 1.0 for u in lane_use)


def test_builds_on_several_host_threads():
    """Four handles built from four host threads at once, each thread on its
    own stream, five builds each (the builds share the pool of page-locked
    blocks through which they read their box counts), equal the same builds run
    one after another, bit for bit.  One lens has a clump of coincident
    particles, so its builds take the full-key sort."""
    import threading

    import paper_1312_1128_amd as g
    import torch

    say("[gpu] builds on several host threads")
    lenses = [synth.nfw_halo(20000 + 5000 * k, 70 + k) for k in range(3)]
    deep = synth.nfw_halo(20000, 74)
    deep.x[:40], deep.y[:40] = deep.x[0], deep.y[0]  # 40 > L + 1 equal keys: a box below level 16
    lenses.append(deep)
    inputs = [(dev(c.x), dev(c.y), dev(c.m), dev(c.s), c.q) for c in lenses]
    torch.cuda.synchronize()
    keys = ("ncells", "max_level", "beg", "end", "next", "leaf", "lbeg", "lend", "M", "cx", "cy", "rcut2", "Q",
            "perm", "key", "list_idx")

    def build_one(t, i):
        x, y, m, s, q = inputs[i]
        return t.build(x, y, m, s, theta=0.3, q=q, leaf_size=8, order=6)

    ref = [build_one(g.Tree(), i).export() for i in range(4)]
    assert ref[3]["max_level"] > 16 and max(r["max_level"] for r in ref[:3]) <= 16
    out, errs = [None] * 4, []

    def worker(i):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                t = g.Tree()
                for _ in range(5):
                    build_one(t, i)
                st.synchronize()
                out[i] = t.export()
        except Exception as e:  # reported after the join
            errs.append(f"lens {i}: {e!r}")

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for i in range(4):
        for k in keys:
            np.testing.assert_array_equal(out[i][k], ref[i][k], err_msg=f"lens {i}: {k}")
