"""Pins of the refinement and interpolation rules (oracle/refine.py) against
what geometry and the linear lens equation fix: the split tiles the parent
square, ranking follows the deflection gradient with ties in cell order, the
(level, i, j) neighbour search equals a brute-force point-in-square search, a
linear deflection field is filled exactly, and tol = 0 fills only exactly
uniform neighbourhoods."""
import numpy as np
import pytest

from oracle import refine


def base_grid(nbase, x0=-0.3, y0=0.1, h0=0.01):
    i, j = np.meshgrid(np.arange(nbase), np.arange(nbase), indexing="xy")
    cx = x0 + (i.ravel() + 0.5) * h0
    cy = y0 + (j.ravel() + 0.5) * h0
    return cx, cy, x0, y0, h0


def test_split_tiles_the_parent_square():
    cx, cy, side = np.zeros(9), np.zeros(9), np.zeros(9)
    cx[0], cy[0], side[0] = 0.2, -0.7, 0.09
    new = refine.split(cx, cy, side, [0], 1)
    assert list(new) == list(range(1, 9))
    assert np.all(side == 0.03)
    # the nine centres form the 3 x 3 lattice of spacing side/3 around the old centre
    pts = sorted(zip(np.round((cx - 0.2) / 0.03, 9), np.round((cy + 0.7) / 0.03, 9)))
    assert pts == sorted((float(a), float(b)) for a in (-1, 0, 1) for b in (-1, 0, 1))
    # row order of the appended cells: dy outer, dx inner
    assert [(round((cx[o] - 0.2) / 0.03), round((cy[o] + 0.7) / 0.03)) for o in new] == refine.RING


def test_rounds_conserve_area_and_keep_cells_disjoint():
    gen = np.random.default_rng(3)
    cx, cy, x0, y0, h0 = base_grid(6)
    cap = 36 + 8 * (4 + 5 + 6)
    X, Y, S = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    X[:36], Y[:36], S[:36] = cx, cy, h0
    n = 36
    for k in (4, 5, 6):
        kap, g1, g2 = gen.normal(size=(3, cap))
        refine.refine_round(X, Y, S, kap, g1, g2, n, k)
        n += 8 * k
        assert np.isclose(np.sum(S[:n] ** 2), (6 * h0) ** 2, rtol=1e-12)
    # every point of a fine probe lattice lies in exactly one cell
    px, py = np.meshgrid(x0 + (np.arange(97) + 0.37) * 6 * h0 / 97, y0 + (np.arange(97) + 0.61) * 6 * h0 / 97)
    inside = (np.abs(px.ravel()[:, None] - X[None, :n]) < S[None, :n] / 2) & \
             (np.abs(py.ravel()[:, None] - Y[None, :n]) < S[None, :n] / 2)
    assert np.all(inside.sum(1) == 1)


def test_rank_follows_the_deflection_gradient_with_ties_in_order():
    """|grad alpha|_F^2 = 2 (kappa^2 + |gamma|^2): the top cells by side |grad alpha|_F."""
    gen = np.random.default_rng(5)
    n = 400
    side = gen.choice([0.01, 0.003, 0.001], n)
    M = gen.normal(size=(n, 2, 2))
    M = 0.5 * (M + M.transpose(0, 2, 1))  # one plane: a symmetric Jacobian
    kap = 0.5 * (M[:, 0, 0] + M[:, 1, 1])
    g1 = 0.5 * (M[:, 0, 0] - M[:, 1, 1])
    g2 = M[:, 0, 1]
    frob = np.sqrt((M ** 2).sum(axis=(1, 2)))
    assert np.allclose(frob ** 2, 2 * (kap ** 2 + g1 ** 2 + g2 ** 2))
    want = side * frob
    top = refine.rank(side, kap, g1, g2, n, 40)
    # the chosen cells are the 40 largest by side |grad alpha| (no near-ties at FP32 here)
    srt = np.sort(want)[::-1]
    assert srt[39] > srt[40] * (1 + 1e-5)
    assert set(top) == set(np.argsort(-want)[:40])
    assert np.all(np.diff(want[top]) <= 0)
    # ties: identical cells keep their index order, wherever they sit
    side[[7, 3, 250, 99]] = 0.02
    kap[7] = 50.0
    for a in (kap, g1, g2):
        a[[3, 250, 99]] = a[7]
    top = refine.rank(side, kap, g1, g2, n, 4)
    assert list(top) == [3, 7, 99, 250]
    # k = 0 ranks nothing, k = n everything
    assert refine.rank(side, kap, g1, g2, n, 0).size == 0
    assert sorted(refine.rank(side, kap, g1, g2, n, n)) == list(range(n))


def brute_neighbour(G, c, dx, dy):
    """The cell whose square holds the centre of the square of c's level next
    to c in direction (dx, dy); -1 outside the base grid."""
    h = G.h0 / 3.0 ** G.lev[c]
    px, py = G.cx[c] + dx * h, G.cy[c] + dy * h
    ext = G.nbase * G.h0
    if not (G.x0 < px < G.x0 + ext and G.y0 < py < G.y0 + ext):
        return -1
    hit = np.nonzero((np.abs(px - G.cx[:G.n]) < G.side[:G.n] / 2) & (np.abs(py - G.cy[:G.n]) < G.side[:G.n] / 2))[0]
    assert hit.size == 1
    return int(hit[0])


def test_neighbour_search_equals_point_in_square():
    gen = np.random.default_rng(7)
    cx, cy, x0, y0, h0 = base_grid(5)
    sched = [3, 4, 6, 9]
    G = refine.NestedGrid(cx, cy, x0, y0, h0, 5, 25 + 8 * sum(sched))
    for k in sched:
        for q in refine.NAMES:
            G.out[q][:G.n] = gen.normal(size=G.n)
        G.interp_round(k, tol=0.0)
    checked = 0
    for c in range(G.n):
        got = G.neighbours(c)
        want = []
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx, dy) == (0, 0):
                    continue
                b = brute_neighbour(G, c, dx, dy)
                if b >= 0 and b != c:
                    want.append(b)
        assert got == want, c
        checked += len(got)
    assert checked > 8 * G.n // 2
    # corner cells of the base grid have 3 neighbours before any split
    G0 = refine.NestedGrid(cx, cy, x0, y0, h0, 5, 25)
    assert len(G0.neighbours(0)) == 3 and len(G0.neighbours(12)) == 8


def linear_field(M, a0, x, y):
    return a0[0] + M[0, 0] * x + M[0, 1] * y, a0[1] + M[1, 0] * x + M[1, 1] * y


@pytest.mark.parametrize("deflections", [False, True])
def test_linear_deflection_field_is_filled_exactly(deflections):
    """alpha = a0 + M x: kappa, gamma are the same in every cell, every cell with
    a neighbour is uniform, and the linear lens equation gives the field's
    value at every new centre.  M symmetric for kappa/gamma; any M from
    deflections alone."""
    M = np.array([[0.31, -0.12], [-0.12, 0.57]]) if not deflections else np.array([[0.31, -0.17], [0.05, 0.62]])
    a0 = np.array([0.2, -0.4])
    kap, g1, g2 = 0.5 * (M[0, 0] + M[1, 1]), 0.5 * (M[0, 0] - M[1, 1]), M[0, 1]
    cx, cy, x0, y0, h0 = base_grid(8)
    sched = [6, 12]
    G = refine.NestedGrid(cx, cy, x0, y0, h0, 8, 64 + 8 * sum(sched))
    n = G.n
    G.out["a1"][:n], G.out["a2"][:n] = linear_field(M, a0, G.cx[:n], G.cy[:n])
    G.out["kappa"][:n], G.out["g1"][:n], G.out["g2"][:n] = kap, g1, g2
    if deflections:
        est = G.estimate_kg(range(n))
        assert np.allclose(est, np.array([kap, g1, g2]) * np.ones((n, 1)), atol=1e-9) or not np.allclose(M, M.T)
    for k in sched:
        n0 = G.n
        order, uni, shoot = G.interp_round(k, tol=1e-6, deflections=deflections)
        assert uni.all() and shoot.size == 0
        new = np.arange(n0, n0 + 8 * k)
        w1, w2 = linear_field(M, a0, G.cx[new], G.cy[new])
        assert np.abs(G.out["a1"][new] - w1).max() < 1e-12 and np.abs(G.out["a2"][new] - w2).max() < 1e-12
        if deflections:
            # A = I - M from three points, so kappa, gamma of the new cells come from M's symmetric part
            want = (1 - (2 - M[0, 0] - M[1, 1]) / 2, ((1 - M[1, 1]) - (1 - M[0, 0])) / 2, (M[1, 0] + M[0, 1]) / 2)
            assert np.allclose(G.out["kappa"][new], want[0], atol=1e-9)
            assert np.allclose(G.out["g1"][new], want[1], atol=1e-9)
            assert np.allclose(G.out["g2"][new], want[2], atol=1e-9)
        else:
            assert np.all(G.out["kappa"][new] == kap) and np.all(G.out["g2"][new] == g2)


def test_tol_zero_fills_only_exactly_uniform_neighbourhoods():
    gen = np.random.default_rng(11)
    cx, cy, x0, y0, h0 = base_grid(6)
    G = refine.NestedGrid(cx, cy, x0, y0, h0, 6, 36 + 8 * 5)
    for q in refine.NAMES:
        G.out[q][:36] = gen.normal(size=36)
    order, uni, shoot = G.interp_round(5, tol=0.0)
    assert not uni.any() and shoot.size == 40
    # the same grid with one constant kappa, gamma: every ranked cell is uniform at tol 0
    G = refine.NestedGrid(cx, cy, x0, y0, h0, 6, 36 + 8 * 5)
    G.out["kappa"][:36], G.out["g1"][:36], G.out["g2"][:36] = 0.3, -0.1, 0.2
    order, uni, shoot = G.interp_round(5, tol=0.0)
    assert uni.all() and shoot.size == 0
    # a single differing neighbour breaks uniformity exactly at its difference
    G = refine.NestedGrid(cx, cy, x0, y0, h0, 6, 36 + 8)
    G.out["kappa"][:36], G.out["g1"][:36], G.out["g2"][:36] = 0.3, -0.1, 0.2
    G.side[14] = 2 * h0  # cell 14 ranks first (its name and square stay those of the base grid)
    G.out["kappa"][15] = 0.3 + 0.25
    assert not G.uniform_kg(14, 0.2499) and G.uniform_kg(14, 0.2501)
