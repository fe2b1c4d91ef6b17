"""Magnification matrix from deflections at three points (App. A) --
TEST INFRASTRUCTURE ONLY (plain Python, FP64).

For a cell centre x_c with deflection alpha_c and two neighbours P, Q, the
offsets u = x_P - x_c, v = x_Q - x_c on the image plane and their images
s = u - (alpha_P - alpha_c), t = v - (alpha_Q - alpha_c) on the source plane
satisfy, to linear order, s = A u and t = A v with
A = [[a11, a21], [a12, a22]] (y_1 = a11 x_1 + a21 x_2, y_2 = a12 x_1 + a22 x_2).
Solving the 4 x 4 system gives, with det = u1 v2 - u2 v1,
    a11 = (v2 s1 - u2 t1)/det,  a21 = (u1 t1 - v1 s1)/det,
    a12 = (v2 s2 - u2 t2)/det,  a22 = (u1 t2 - v1 s2)/det.
A cell is tested with every pair of its neighbours that is not collinear
with the centre (reading: |det| > 1e-6 |u| |v|); it is uniform when each
element of A agrees over all pairs within the tolerance.
"""
from __future__ import annotations

import math


def three_point(xc, yc, ac1, ac2, nbrs):
    """nbrs: [(x, y, alpha1, alpha2), ...] in the order the neighbours are
    located.  Returns (npairs, mins, maxs, sums) over the pair estimates of
    (a11, a21, a12, a22)."""
    mn, mx, sm = [math.inf] * 4, [-math.inf] * 4, [0.0] * 4
    npairs = 0
    for p in range(len(nbrs)):
        for q in range(p + 1, len(nbrs)):
            xp, yp, ap1, ap2 = (float(v) for v in nbrs[p])
            xq, yq, aq1, aq2 = (float(v) for v in nbrs[q])
            u1, u2, v1, v2 = xp - xc, yp - yc, xq - xc, yq - yc
            s1, s2 = u1 - (ap1 - ac1), u2 - (ap2 - ac2)
            t1, t2 = v1 - (aq1 - ac1), v2 - (aq2 - ac2)
            det = u1 * v2 - u2 * v1
            if not (abs(det) > 1e-6 * math.sqrt((u1 * u1 + u2 * u2) * (v1 * v1 + v2 * v2))):
                continue
            e = ((v2 * s1 - u2 * t1) / det, (u1 * t1 - v1 * s1) / det, (v2 * s2 - u2 * t2) / det,
                 (u1 * t2 - v1 * s2) / det)
            for k in range(4):
                mn[k] = min(mn[k], e[k])
                mx[k] = max(mx[k], e[k])
                sm[k] = sm[k] + e[k]
            npairs += 1
    return npairs, mn, mx, sm


def uniform(npairs, mn, mx, tol):
    return npairs > 0 and all(mx[k] - mn[k] <= tol for k in range(4))


def mean_A(npairs, sm):
    return [s / npairs for s in sm] if npairs > 0 else [0.0, 0.0, 0.0, 0.0]


def kappa_gamma(A):
    """kappa = 1 - (a11 + a22)/2, gamma1 = (a22 - a11)/2, gamma2 = -(a12 + a21)/2
    (A = I - [[kappa + g1, g2], [g2, kappa - g1]] for one plane)."""
    a11, a21, a12, a22 = A
    return 1.0 - 0.5 * (a11 + a22), 0.5 * (a22 - a11), -0.5 * (a12 + a21)
