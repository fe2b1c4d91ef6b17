"""Pins of the oracle adjoints (gradients of L = sum_r g_r . alpha_r with
respect to particle masses, positions and smoothing lengths).

* Central finite differences of the forward oracles (brute force, and the
  tree with its decisions frozen) -- an independent route to the same numbers.
* Exact identities of the lensing sums: alpha is homogeneous of degree one in
  the masses (Euler), depends on ray - particle only (translation), and is
  scale covariant (x -> lambda x, s -> lambda s, m -> lambda^2 m).
"""
import numpy as np
import pytest

import synth


def lens_and_rays(n=120, nr=60, seed=201):
    lens = synth.gaussian_blobs(n, seed, s_lo=0.02, s_hi=0.3)
    g = synth.rng(seed + 1)
    lens.s[g.random(n) < 0.25] = 0.0
    px, py = synth.uniform_points(nr, seed + 2)
    ga = g.normal(size=(nr, 2))
    return lens, px, py, ga


def loss_direct(ora, lens, x, y, m, s, px, py, ga):
    A = ora.direct(x, y, m, s, lens.q, px, py)
    return float(np.sum(A[:, 0] * ga[:, 0] + A[:, 1] * ga[:, 1]))


def test_direct_grad_matches_finite_differences(ora):
    lens, px, py, ga = lens_and_rays()
    dm, dx, dy, ds = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga)
    g = synth.rng(5)
    for i in g.choice(lens.n, 12, replace=False):
        for name, arr, grad, h in [("m", lens.m, dm, 1e-7), ("x", lens.x, dx, 1e-7),
                                   ("y", lens.y, dy, 1e-7), ("s", lens.s, ds, 1e-7)]:
            if name == "s" and lens.s[i] == 0:
                continue
            p = {"x": lens.x.copy(), "y": lens.y.copy(), "m": lens.m.copy(), "s": lens.s.copy()}
            p[name][i] = arr[i] + h
            lp = loss_direct(ora, lens, p["x"], p["y"], p["m"], p["s"], px, py, ga)
            p[name][i] = arr[i] - h
            lm = loss_direct(ora, lens, p["x"], p["y"], p["m"], p["s"], px, py, ga)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-5 * max(abs(grad[i]), 1e-3 * np.abs(grad).max()), (name, i)


@pytest.mark.parametrize("theta,order", [(0.5, 3), (0.3, 6)])
def test_tree_grad_matches_frozen_finite_differences(ora, theta, order):
    lens, px, py, ga = lens_and_rays(300, 80, 211)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, 4, order)
    _, cnt = T.shoot(px, py, counts=True)
    assert cnt[:, 1].sum() > 0
    dm, dx, dy, ds = T.grad(px, py, ga)
    T.record(px, py)
    g = synth.rng(6)
    base = {"x": lens.x, "y": lens.y, "m": lens.m, "s": lens.s}
    grads = {"x": dx, "y": dy, "m": dm, "s": ds}
    for i in g.choice(lens.n, 15, replace=False):
        for name in ["m", "x", "y", "s"]:
            if name == "s" and lens.s[i] == 0:
                continue
            h = 1e-6
            vals = []
            for sgn in (1, -1):
                p = {k: v.copy() for k, v in base.items()}
                p[name][i] += sgn * h
                T.set_particles(p["x"], p["y"], p["m"], p["s"])
                B = T.shoot_frozen(px, py)
                vals.append(np.sum(B[:, 0] * ga[:, 0] + B[:, 1] * ga[:, 1]))
            fd = (vals[0] - vals[1]) / (2 * h)
            gr = grads[name][i]
            assert abs(fd - gr) <= 1e-5 * max(abs(gr), 1e-3 * np.abs(grads[name]).max()), (name, i, fd, gr)
    T.set_particles(lens.x, lens.y, lens.m, lens.s)


def test_tree_grad_theta_zero_is_direct_grad(ora):
    lens, px, py, ga = lens_and_rays(200, 50, 221)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.0, 3, 2)
    a = T.grad(px, py, ga)
    b = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-10, atol=1e-12 * np.abs(v).max())


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_grad_identities(ora, theta):
    lens, px, py, ga = lens_and_rays(300, 70, 231)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, 4, 4)
    B = T.shoot(px, py)
    dm, dx, dy, ds = T.grad(px, py, ga)
    # Euler: sum_i m_i dL/dm_i = L
    L = np.sum(B[:, 0] * ga[:, 0] + B[:, 1] * ga[:, 1])
    assert abs(np.sum(lens.m * dm) - L) < 1e-10 * np.sum(np.abs(lens.m * dm))
    # translation: sum_i dL/dx_i = -sum_r (J_r g_r)
    k, g1, g2 = B[:, 2], B[:, 3], B[:, 4]
    tx = -np.sum((k + g1) * ga[:, 0] + g2 * ga[:, 1])
    ty = -np.sum(g2 * ga[:, 0] + (k - g1) * ga[:, 1])
    sc = np.sum(np.abs(dx)) + np.sum(np.abs(dy))
    assert abs(np.sum(dx) - tx) < 1e-10 * sc
    assert abs(np.sum(dy) - ty) < 1e-10 * sc
    # scale covariance: sum_i (x_i dL/dx_i + y_i dL/dy_i + s_i dL/ds_i + 2 m_i dL/dm_i)
    #   = sum_r g_r . (alpha_r - J_r x_r)   [alpha(lambda x) = lambda alpha(x)]
    lhs = np.sum(lens.x * dx + lens.y * dy + lens.s * ds + 2 * lens.m * dm)
    jx1 = (k + g1) * px + g2 * py
    jx2 = g2 * px + (k - g1) * py
    rhs = np.sum(ga[:, 0] * (B[:, 0] - jx1) + ga[:, 1] * (B[:, 1] - jx2))
    assert abs(lhs - rhs) < 1e-9 * (np.sum(np.abs(lens.x * dx)) + np.sum(np.abs(lens.m * dm)))


# ------------------------------------------------ kappa and gamma cotangents

def test_unit_dterms_match_finite_differences(ora):
    """d(kappa, gamma)/d(offset) and d/ds of one particle, against central
    differences of its pinned kappa and gamma."""
    q, s = 3.0, 0.2
    for (d1, d2) in [(0.013, -0.02), (0.1, 0.07), (-0.25, 0.31), (0.5, 0.45), (0.9, -0.2)]:
        for sm in (s, 0.0):
            inside = sm > 0 and d1 * d1 + d2 * d2 < (q * sm) ** 2
            dt = ora.unit_dterms(d1, d2, sm, q, inside)
            h = 1e-6
            fx = (ora.unit_terms(d1 + h, d2, sm, q, inside) - ora.unit_terms(d1 - h, d2, sm, q, inside)) / (2 * h)
            fy = (ora.unit_terms(d1, d2 + h, sm, q, inside) - ora.unit_terms(d1, d2 - h, sm, q, inside)) / (2 * h)
            ref = np.array([fx[2], fy[2], fx[3], fy[3], fx[4], fy[4]])
            sc = np.abs(ref).max()
            np.testing.assert_allclose(dt[:6], ref, rtol=1e-6, atol=1e-8 * sc)
            if inside:
                fs = (ora.unit_terms(d1, d2, sm + h, q, True) - ora.unit_terms(d1, d2, sm - h, q, True)) / (2 * h)
                np.testing.assert_allclose(dt[6:], fs[2:5], rtol=1e-6, atol=1e-8 * np.abs(fs[2:5]).max())
            else:
                assert np.all(dt[6:] == 0.0)
    # the point mass: kappa = 0 everywhere, |d gamma| = 2 / r^3
    dt = ora.unit_dterms(0.3, 0.4, 0.0, q, False)
    assert dt[0] == dt[1] == 0.0
    assert np.hypot(dt[2], dt[3]) == pytest.approx(2 / 0.5 ** 3, rel=1e-12)


def full_loss(A, ga, gk, gg):
    return float(np.sum(A[:, 0] * ga[:, 0] + A[:, 1] * ga[:, 1] + A[:, 2] * gk + A[:, 3] * gg[:, 0]
                        + A[:, 4] * gg[:, 1]))


def cotangents(nr, seed):
    g = synth.rng(seed)
    return g.normal(size=nr), g.normal(size=(nr, 2))


def test_direct_grad_kappa_gamma_matches_finite_differences(ora):
    lens, px, py, ga = lens_and_rays(100, 60, 241)
    gk, gg = cotangents(px.size, 242)
    dm, dx, dy, ds = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga, gk=gk, gg=gg)
    g = synth.rng(7)
    base = {"x": lens.x, "y": lens.y, "m": lens.m, "s": lens.s}
    grads = {"x": dx, "y": dy, "m": dm, "s": ds}
    for i in g.choice(lens.n, 12, replace=False):
        for name in ["m", "x", "y", "s"]:
            if name == "s" and lens.s[i] == 0:
                continue
            h, vals = 1e-7, []
            for sgn in (1, -1):
                p = {k: v.copy() for k, v in base.items()}
                p[name][i] += sgn * h
                vals.append(full_loss(ora.direct(p["x"], p["y"], p["m"], p["s"], lens.q, px, py), ga, gk, gg))
            fd = (vals[0] - vals[1]) / (2 * h)
            gr = grads[name][i]
            assert abs(fd - gr) <= 1e-5 * max(abs(gr), 1e-3 * np.abs(grads[name]).max()), (name, i, fd, gr)
    # alpha-only cotangents reproduce the alpha gradient
    a = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga)
    b = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga, gk=0 * gk, gg=0 * gg)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("theta,order", [(0.5, 3), (0.3, 6)])
def test_tree_grad_kappa_gamma_matches_frozen_finite_differences(ora, theta, order):
    lens, px, py, ga = lens_and_rays(300, 80, 251)
    gk, gg = cotangents(px.size, 252)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, theta, 4, order)
    _, cnt = T.shoot(px, py, counts=True)
    assert cnt[:, 1].sum() > 0 and cnt[:, 4].sum() > 0
    dm, dx, dy, ds = T.grad(px, py, ga, gk=gk, gg=gg)
    T.record(px, py)
    g = synth.rng(8)
    base = {"x": lens.x, "y": lens.y, "m": lens.m, "s": lens.s}
    grads = {"x": dx, "y": dy, "m": dm, "s": ds}
    for i in g.choice(lens.n, 15, replace=False):
        for name in ["m", "x", "y", "s"]:
            if name == "s" and lens.s[i] == 0:
                continue
            h, vals = 1e-6, []
            for sgn in (1, -1):
                p = {k: v.copy() for k, v in base.items()}
                p[name][i] += sgn * h
                T.set_particles(p["x"], p["y"], p["m"], p["s"])
                vals.append(full_loss(T.shoot_frozen(px, py), ga, gk, gg))
            fd = (vals[0] - vals[1]) / (2 * h)
            gr = grads[name][i]
            assert abs(fd - gr) <= 1e-5 * max(abs(gr), 1e-3 * np.abs(grads[name]).max()), (name, i, fd, gr)
    T.set_particles(lens.x, lens.y, lens.m, lens.s)
    # Euler: every output is linear in the masses
    B = T.shoot(px, py)
    assert abs(np.sum(lens.m * dm) - full_loss(B, ga, gk, gg)) < 1e-10 * np.sum(np.abs(lens.m * dm))


def test_tree_grad_kappa_gamma_theta_zero_is_direct(ora):
    lens, px, py, ga = lens_and_rays(200, 50, 261)
    gk, gg = cotangents(px.size, 262)
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, lens.q, 0.0, 3, 2)
    a = T.grad(px, py, ga, gk=gk, gg=gg)
    b = ora.direct_grad(lens.x, lens.y, lens.m, lens.s, lens.q, px, py, ga, gk=gk, gg=gg)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-10, atol=1e-12 * np.abs(v).max())
