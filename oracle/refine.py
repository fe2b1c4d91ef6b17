"""Adaptive grid refinement (Sec. 4) and its interpolation shortcut (Sec. 3.4,
App. A) -- TEST INFRASTRUCTURE ONLY (plain Python and numpy).

The image plane is covered by square cells, each with one ray shot at its
centre.  A refinement round ranks the cells by how fast the deflection varies
across them and splits the top ones 3 x 3: the cell keeps its centre ray and
becomes the middle ninth, and 8 new cells (new rays) are added around it.

Readings taken (the paper gives the rules in words only):
* rank by side^2 (kappa^2 + gamma1^2 + gamma2^2), which is monotone in
  side |grad alpha|_F since |grad alpha|_F^2 = 2 (kappa^2 + |gamma|^2) for one
  plane; the score is formed in FP32 as the library forms it, because it
  decides an integer (which cells are split); ties go to the lower index;
* the new cells of a split are appended 8 per split cell, in rank order,
  each in row order (dy = -1, 0, 1 outer, dx = -1, 0, 1 inner, centre skipped);
* cells form a nested grid: a base grid of nbase x nbase cells of side h0
  from (x0, y0) is level 0, and a split cell's ninths are one level deeper, so
  a cell is named by (level, i, j) with centre x0 + (i + 1/2) h0 / 3^level;
* the neighbours of a cell are, on each of its 8 sides, the cell of the same
  level there, else the coarser cell covering that spot (none outside the
  base grid).  A cell that was split keeps answering for its old name: its
  centre ray is still the centre of that square;
* interpolation (Sec. 3.4): before a ranked cell is split it is "uniform" if
  it has at least one neighbour and every neighbour's kappa, gamma1, gamma2
  differ from its own by at most tol (FP32 differences, as the library takes
  them).  The 8 new cells of a uniform cell are not shot: they get the linear
  lens equation's alpha = alpha_c + (I - A_c)(x - x_c) with
  I - A_c = [[kappa + gamma1, gamma2], [gamma2, kappa - gamma1]], and the
  cell's kappa, gamma;
* without kappa and gamma (deflection-only walks) the magnification matrix
  comes from deflections at three points (App. A, ``oracle.interp``): the cell
  is uniform if it has a non-collinear pair of neighbours and every element of
  the pair estimates of A agrees within tol; the new cells then use the mean
  estimate, alpha = alpha_c + (I - A)(x - x_c), kappa = 1 - (a11 + a22)/2,
  gamma1 = (a22 - a11)/2, gamma2 = -(a12 + a21)/2.

This module shares nothing with the GPU library.
"""
from __future__ import annotations

import numpy as np

from . import interp

NAMES = ("a1", "a2", "kappa", "g1", "g2")
# offsets of the 8 new cells of a split, in the order they are appended
RING = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy) != (0, 0)]


def score32(side, kappa, g1, g2) -> np.ndarray:
    """side^2 (kappa^2 + gamma1^2 + gamma2^2) in FP32 (NaN scores as 0)."""
    f = np.float32
    h = np.asarray(side).astype(f)
    k, a, b = (np.asarray(v).astype(f) for v in (kappa, g1, g2))
    with np.errstate(over="ignore", invalid="ignore"):
        sc = (h * h) * ((k * k + a * a) + b * b)
    return np.where(np.isnan(sc), f(0), sc).astype(f)


def rank(side, kappa, g1, g2, n: int, k: int) -> np.ndarray:
    """Indices of the k cells among the first n with the largest score, best
    first; equal scores in increasing index order."""
    sc = score32(side[:n], kappa[:n], g1[:n], g2[:n]).astype(np.float64)
    order = np.lexsort((np.arange(n), -sc))
    return order[:k]


def split(cx, cy, side, order, n: int):
    """Split the cells `order` 3 x 3 in place: each becomes the middle ninth and
    8 cells are appended at n + 8 t + q.  Returns the indices appended."""
    new = []
    for t, c in enumerate(order):
        h3 = side[c] / 3.0
        for q, (dx, dy) in enumerate(RING):
            o = n + 8 * t + q
            cx[o] = cx[c] + float(dx) * h3
            cy[o] = cy[c] + float(dy) * h3
            side[o] = h3
            new.append(o)
        side[c] = h3
    return np.array(new, dtype=np.int64)


def refine_round(cx, cy, side, kappa, g1, g2, n: int, k: int) -> np.ndarray:
    """One round without interpolation: rank, then split.  Returns the ranked cells."""
    order = rank(side, kappa, g1, g2, n, k)
    split(cx, cy, side, order, n)
    return order


class NestedGrid:
    """The cells of a refined base grid with their (level, i, j) names and a
    name -> cell table, plus their ray outputs (FP64 copies)."""

    def __init__(self, cx, cy, x0: float, y0: float, h0: float, nbase: int, capacity: int):
        n = len(cx)
        self.x0, self.y0, self.h0, self.nbase = float(x0), float(y0), float(h0), int(nbase)
        self.n = n
        self.cx = np.zeros(capacity)
        self.cy = np.zeros(capacity)
        self.side = np.zeros(capacity)
        self.cx[:n], self.cy[:n], self.side[:n] = cx, cy, h0
        self.lev = np.zeros(capacity, np.int64)
        self.ci = np.zeros(capacity, np.int64)
        self.cj = np.zeros(capacity, np.int64)
        self.ci[:n] = np.floor((self.cx[:n] - x0) / h0).astype(np.int64)
        self.cj[:n] = np.floor((self.cy[:n] - y0) / h0).astype(np.int64)
        self.table = {(0, int(i), int(j)): c for c, (i, j) in enumerate(zip(self.ci[:n], self.cj[:n]))}
        self.out = {q: np.zeros(capacity) for q in NAMES}

    def locate(self, level: int, i: int, j: int) -> int:
        """The cell named (level, i, j), else the nearest coarser cell whose
        square holds that spot; -1 outside the base grid."""
        for l in range(level, -1, -1):
            span = 3 ** l
            if i < 0 or j < 0 or i >= self.nbase * span or j >= self.nbase * span:
                return -1
            c = self.table.get((l, i, j), -1)
            if c >= 0:
                return c
            i, j = i // 3, j // 3
        return -1

    def neighbours(self, c: int) -> list:
        out = []
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0:
                    continue
                nb = self.locate(int(self.lev[c]), int(self.ci[c]) + dx, int(self.cj[c]) + dy)
                if nb >= 0 and nb != c:
                    out.append(nb)
        return out

    def _split_names(self, order, n):
        for t, c in enumerate(order):
            l, i, j = int(self.lev[c]) + 1, 3 * int(self.ci[c]) + 1, 3 * int(self.cj[c]) + 1
            for q, (dx, dy) in enumerate(RING):
                o = n + 8 * t + q
                self.lev[o], self.ci[o], self.cj[o] = l, i + dx, j + dy
                self.table[(l, i + dx, j + dy)] = o
            self.lev[c], self.ci[c], self.cj[c] = l, i, j
            self.table[(l, i, j)] = int(c)

    def uniform_kg(self, c: int, tol: float) -> bool:
        """kappa, gamma of every neighbour within tol of the cell's (FP32)."""
        f = np.float32
        nb = self.neighbours(c)
        if not nb:
            return False
        for q in ("kappa", "g1", "g2"):
            for b in nb:
                if not abs(f(self.out[q][b]) - f(self.out[q][c])) <= f(tol):
                    return False
        return True

    def three_point(self, c: int):
        nb = self.neighbours(c)
        o = self.out
        return interp.three_point(self.cx[c], self.cy[c], o["a1"][c], o["a2"][c],
                                  [(self.cx[b], self.cy[b], o["a1"][b], o["a2"][b]) for b in nb])

    def estimate_kg(self, cells) -> np.ndarray:
        """kappa, gamma1, gamma2 of the cells from their mean three-point A (0 without a pair)."""
        res = np.zeros((len(cells), 3))
        for t, c in enumerate(cells):
            npairs, _, _, sm = self.three_point(c)
            res[t] = interp.kappa_gamma(interp.mean_A(npairs, sm)) if npairs > 0 else (0.0, 0.0, 0.0)
        return res

    def interp_round(self, k: int, tol: float, deflections: bool = False):
        """One refinement round with the interpolation shortcut on the first
        self.n cells.  Fills the new cells of uniform cells; returns (ranked
        cells, their uniform flags, the new cells left to shoot)."""
        n = self.n
        o = self.out
        order = rank(self.side, o["kappa"], o["g1"], o["g2"], n, k)
        if deflections:
            tests = [self.three_point(c) for c in order]
            tol64 = float(np.float32(tol))
            uni = [interp.uniform(t[0], t[1], t[2], tol64) for t in tests]
        else:
            uni = [self.uniform_kg(c, tol) for c in order]
        new = split(self.cx, self.cy, self.side, order, n)
        self._split_names(order, n)
        shoot = []
        for t, c in enumerate(order):
            if deflections:
                A = interp.mean_A(tests[t][0], tests[t][3])
                a11, a21, a12, a22 = A
                M = ((1.0 - a11, -a21), (-a12, 1.0 - a22))  # I - A
                kg = interp.kappa_gamma(A)
            else:
                kap, g1, g2 = o["kappa"][c], o["g1"][c], o["g2"][c]
                M = ((kap + g1, g2), (g2, kap - g1))
                kg = (kap, g1, g2)
            for q in range(8):
                b = new[8 * t + q]
                if not uni[t]:
                    shoot.append(int(b))
                    continue
                ux, uy = self.cx[b] - self.cx[c], self.cy[b] - self.cy[c]
                o["a1"][b] = o["a1"][c] + M[0][0] * ux + M[0][1] * uy
                o["a2"][b] = o["a2"][c] + M[1][0] * ux + M[1][1] * uy
                o["kappa"][b], o["g1"][b], o["g2"][b] = kg
        self.n = n + 8 * k
        return order, np.array(uni, dtype=bool), np.array(shoot, dtype=np.int64)
