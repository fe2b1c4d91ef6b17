"""Pins of the three-point magnification matrix (App. A): exact for a linear
deflection field (any matrix, not only a symmetric one), collinear pairs
skipped, and the spread of the pair estimates measuring the departure from
linearity."""
import math

import numpy as np

from oracle import interp


def grid_neighbours(xc, yc, h, field, coarse=None):
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            x, y = xc + dx * h, yc + dy * h
            if coarse and (dx, dy) in coarse:
                x, y = coarse[(dx, dy)]
            a1, a2 = field(x, y)
            out.append((x, y, a1, a2))
    return out


def test_linear_field_is_recovered_exactly():
    M = np.array([[0.31, -0.17], [0.05, 0.62]])  # d alpha_i / d x_j, not symmetric
    a0 = np.array([0.2, -0.4])
    field = lambda x, y: tuple(a0 + M @ np.array([x, y]))
    xc, yc, h = 0.3, -0.1, 1e-3
    ac = field(xc, yc)
    # a neighbour replaced by the centre of a coarser cell (an off-grid direction)
    nb = grid_neighbours(xc, yc, h, field, coarse={(1, 1): (xc + 2.5 * h, yc + 1.5 * h)})
    n, mn, mx, sm = interp.three_point(xc, yc, ac[0], ac[1], nb)
    assert n > 20
    A = interp.mean_A(n, sm)
    ref = [1 - M[0, 0], -M[0, 1], -M[1, 0], 1 - M[1, 1]]  # a11, a21, a12, a22 of A = I - M
    for k in range(4):
        assert abs(A[k] - ref[k]) < 1e-9 and mx[k] - mn[k] < 1e-9, k
    assert interp.uniform(n, mn, mx, 1e-8)
    # for one plane (symmetric M) kappa and gamma come back
    S = np.array([[0.3, 0.1], [0.1, 0.5]])
    field2 = lambda x, y: tuple(S @ np.array([x, y]))
    nb = grid_neighbours(xc, yc, h, field2)
    n, mn, mx, sm = interp.three_point(xc, yc, *field2(xc, yc), nb)
    k, g1, g2 = interp.kappa_gamma(interp.mean_A(n, sm))
    # I - A = [[k + g1, g2], [g2, k - g1]] = S
    assert abs(k - 0.4) < 1e-9 and abs(g1 - (-0.1)) < 1e-9 and abs(g2 - 0.1) < 1e-9


def test_collinear_neighbours_give_no_pair():
    field = lambda x, y: (0.1 * x, 0.2 * y)
    nb = [(0.1 * t, 0.0) + field(0.1 * t, 0.0) for t in (-2, -1, 1, 3)]
    assert interp.three_point(0.0, 0.0, 0.0, 0.0, nb)[0] == 0
    assert not interp.uniform(0, [0] * 4, [0] * 4, 1.0)


def test_spread_measures_curvature():
    """For alpha = grad of a quadratic plus a cubic term the pair estimates
    differ by O(h |grad A|): the test passes for a large tolerance only."""
    c3 = 0.8
    field = lambda x, y: (0.2 * x + c3 * x * x, 0.3 * y)
    xc, yc = 0.1, 0.2
    for h in (1e-2, 1e-3):
        nb = grid_neighbours(xc, yc, h, field)
        n, mn, mx, sm = interp.three_point(xc, yc, *field(xc, yc), nb)
        spread = max(mx[k] - mn[k] for k in range(4))
        assert 0.5 * c3 * h < spread < 8 * c3 * h  # O(h) in h
        assert interp.uniform(n, mn, mx, 10 * c3 * h) and not interp.uniform(n, mn, mx, 0.1 * c3 * h)
        assert math.isclose(interp.mean_A(n, sm)[0], 1 - (0.2 + 2 * c3 * xc), rel_tol=0, abs_tol=4 * c3 * h)
