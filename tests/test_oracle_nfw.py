"""Pins of the truncated-NFW halo oracle (halos as "particles", Sec. 3.2;
the paper's halo convergence test of Sec. 5.1)."""
import numpy as np
import pytest

import synth


def F_direct(x):
    return np.arccosh(1 / x) / np.sqrt(1 - x * x) if x < 1 else np.arccos(1 / x) / np.sqrt(x * x - 1)


def test_shape_functions(ora):
    from scipy.integrate import quad

    for x in (0.05, 0.3, 0.9, 0.97, 1.03, 1.5, 3.0, 8.0):
        assert abs(ora.nfw_F(x) - F_direct(x)) <= 1e-13 * F_direct(x), x
    # both sides of the series switch near x = 1
    for e in (-1.01e-2, -0.99e-2, 0.99e-2, 1.01e-2):
        x = np.sqrt(1 + e)
        assert abs(ora.nfw_F(x) - F_direct(x)) <= 2e-13, e
    assert ora.nfw_f(1.0) == pytest.approx(1 / 3, rel=1e-15)
    # g is the enclosed-mass shape: g(x) = integral_0^x t f(t) dt, g' = x f
    for x in (2e-4, 1e-3, 0.02, 0.5, 0.999, 1.0, 1.001, 2.0, 3.0):
        ref = quad(lambda t: t * ora.nfw_f(t), 0, x, limit=400, epsabs=1e-30, epsrel=1e-12)[0]
        assert abs(ora.nfw_g(x) - ref) <= 1e-10 * ref, x
        h = 1e-6 * x
        dg = (ora.nfw_g(x + h) - ora.nfw_g(x - h)) / (2 * h)
        assert abs(dg - x * ora.nfw_f(x)) <= 1e-7 * x * ora.nfw_f(x), x


def test_shapes_near_one_against_series():
    """Around x = 1, F = sum (-e)^k / (2k + 1) and f = (1 - F) / e =
    sum (-e)^k / (2k + 3) with e = x^2 - 1 (the Taylor series of atan(y)/y
    and atanh(y)/y in y^2 = +-e), summed in 50-digit decimal arithmetic for the
    exact binary x: both sides of the series switch and the closed forms just
    beyond it, where F's digits cancel in f."""
    from decimal import Decimal, getcontext

    import oracle as ora

    getcontext().prec = 50
    for x in (0.9, 0.95, 0.994, 0.99499, 0.995, 0.999, 0.9999, 1.0, 1.0001, 1.001, 1.00499, 1.005, 1.006, 1.05, 1.1):
        e = Decimal(x) * Decimal(x) - 1
        F = f = Decimal(0)
        p = Decimal(1)
        for k in range(400):
            F += p / (2 * k + 1)
            f += p / (2 * k + 3)
            p *= -e
        assert abs(ora.nfw_F(x) - float(F)) <= 4e-16 * float(F), x
        assert abs(ora.nfw_f(x) - float(f)) <= 1e-13 * float(f), x


@pytest.mark.parametrize("r_over_R", [0.001, 0.1, 0.33, 0.5, 0.9, 1.2])
def test_kappa_gamma_from_alpha(ora, r_over_R):
    R, c, phi = 0.3, 3.0, 0.4
    r = r_over_R * R
    d1, d2 = r * np.cos(phi), r * np.sin(phi)

    def a(u, v):
        return ora.nfw_terms(u, v, R, c, u * u + v * v < R * R)[:2]

    h = 1e-6 * r
    dx = (a(d1 + h, d2) - a(d1 - h, d2)) / (2 * h)
    dy = (a(d1, d2 + h) - a(d1, d2 - h)) / (2 * h)
    t = ora.nfw_terms(d1, d2, R, c, r < R)
    scale = np.abs([dx, dy]).max()
    assert abs(0.5 * (dx[0] + dy[1]) - t[2]) <= 1e-6 * scale  # kappa = div(alpha) / 2
    assert abs(0.5 * (dx[0] - dy[1]) - t[3]) <= 1e-6 * scale  # gamma1
    assert abs(dx[1] - t[4]) <= 1e-6 * scale and abs(dy[0] - t[4]) <= 1e-6 * scale  # gamma2, curl-free


def test_mass_and_continuity(ora):
    from scipy.integrate import quad

    R, c = 0.2, 3.0
    mass = quad(lambda r: 2 * np.pi * r * ora.nfw_terms(r, 0.0, R, c, True)[2], 0, R, limit=400,
                epsabs=1e-14, epsrel=1e-11)[0]
    assert mass == pytest.approx(np.pi, rel=1e-9)  # integral of kappa = pi m (m in units of pi Sigma_crit)
    inner = ora.nfw_terms(R * (1 - 1e-13), 0.0, R, c, True)
    outer = ora.nfw_terms(R * (1 + 1e-13), 0.0, R, c, False)
    assert abs(inner[0] - outer[0]) <= 1e-10 * outer[0]  # alpha continuous; a point mass outside


def test_halo_field_kappa_exact_for_any_theta(ora):
    """The paper's halo test: kappa from halos intersecting the ray only, so
    the tree's kappa has no error at any theta; alpha and gamma converge."""
    lens, c = synth.nfw_halo_field(3000, 97)
    rx, ry = synth.uniform_points(200, 98, -0.8, 0.8)
    rx[:4], ry[:4] = [0.0, 1e-3, -0.01, 0.02], [0.0, 2e-3, 0.005, -0.01]
    ref = ora.direct_nfw(lens.x, lens.y, lens.m, lens.s, c, rx, ry)
    T0 = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, 0.0, 8, 4, nfw=True)
    np.testing.assert_allclose(T0.shoot(rx, ry), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    prev = None
    for theta in (0.5, 0.3, 0.1):
        got = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, theta, 8, 4, nfw=True).shoot(rx, ry)
        assert np.abs(got[:, 2] - ref[:, 2]).max() <= 1e-12 * np.abs(ref[:, 2]).max()
        ea = (np.linalg.norm(got[:, :2] - ref[:, :2], axis=1) / np.linalg.norm(ref[:, :2], axis=1)).max()
        if prev is not None:
            assert ea < prev
        prev = ea
    assert prev < 1e-6


def test_potential_H_is_the_integral_of_g_over_x(ora):
    """psi of a halo uses H with H' = g(x)/x (alpha = grad psi, Sec. 3.2)."""
    from scipy.integrate import quad

    for x in (1e-3, 0.05, 0.5, 0.99, 1.0, 1.01, 2.0, 5.0):
        ref = quad(lambda t: ora.nfw_g(t) / t, 0.7, x, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
        assert abs((ora.nfw_H(x) - ora.nfw_H(0.7)) - ref) <= 1e-11 * max(1.0, abs(ref)), x


@pytest.mark.parametrize("r_over_R", [0.002, 0.1, 0.33, 0.7, 0.99, 1.4])
def test_potential_gradient_and_laplacian(ora, r_over_R):
    R, c, phi = 0.3, 3.0, 0.7
    r = r_over_R * R
    d1, d2 = r * np.cos(phi), r * np.sin(phi)

    def psi(u, v):
        return ora.nfw_psi(u, v, R, c, u * u + v * v < R * R)

    # central differences: truncation ~ (h/r)^2 relative, rounding ~ eps |psi| / h
    h = 1e-4 * r
    g1 = (psi(d1 + h, d2) - psi(d1 - h, d2)) / (2 * h)
    g2 = (psi(d1, d2 + h) - psi(d1, d2 - h)) / (2 * h)
    t = ora.nfw_terms(d1, d2, R, c, r < R)
    an = np.hypot(t[0], t[1])
    assert abs(g1 - t[0]) <= 1e-6 * an and abs(g2 - t[1]) <= 1e-6 * an
    h = 1e-3 * r
    lap = (psi(d1 + h, d2) + psi(d1 - h, d2) + psi(d1, d2 + h) + psi(d1, d2 - h) - 4 * psi(d1, d2)) / (h * h)
    # Poisson: laplacian psi = 2 kappa; the 5-point stencil errs by ~ (h/r)^2 / r^2
    assert abs(lap - 2 * t[2]) <= 1e-4 * 2 * t[2] + 1e-4 / (r * r)


def test_potential_continuity_and_tree(ora):
    R, c = 0.25, 3.0
    inner = ora.nfw_psi(R * (1 - 1e-13), 0.0, R, c, True)
    outer = ora.nfw_psi(R * (1 + 1e-13), 0.0, R, c, False)
    assert abs(inner - outer) <= 1e-12 and abs(outer - np.log(R)) <= 1e-12
    lens, c = synth.nfw_halo_field(2000, 131)
    rx, ry = synth.uniform_points(300, 132, -0.9, 0.9)
    ref = ora.direct_nfw_psi(lens.x, lens.y, lens.m, lens.s, c, rx, ry)
    T0 = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, 0.0, 8, 4, nfw=True)
    np.testing.assert_allclose(T0.shoot_psi(rx, ry), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    got = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, 0.3, 8, 8, nfw=True).shoot_psi(rx, ry)
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def test_derivative_shapes_and_terms(ora):
    """f'(x) and the per-unit-mass derivatives of alpha, kappa, gamma by the
    offset and by the size R (the adjoint's terms), against central
    differences of the pinned shapes and terms."""
    for x in (0.02, 0.4, 0.93, 0.995, 1.0, 1.004, 1.2, 4.0):
        h = 1e-6 * x
        fd = (ora.nfw_f(x + h) - ora.nfw_f(x - h)) / (2 * h)
        assert abs(ora.nfw_df(x) - fd) <= 1e-6 * abs(fd) + 1e-9, x
    R, c = 0.3, 3.0
    for (d1, d2) in [(0.004, -0.002), (0.05, 0.03), (-0.09, 0.1), (0.2, -0.15), (0.29, 0.01), (0.4, 0.2)]:
        inside = d1 * d1 + d2 * d2 < R * R
        dt = ora.nfw_dterms(d1, d2, R, c, inside)
        h = 1e-7
        fx = (ora.nfw_terms(d1 + h, d2, R, c, inside) - ora.nfw_terms(d1 - h, d2, R, c, inside)) / (2 * h)
        fy = (ora.nfw_terms(d1, d2 + h, R, c, inside) - ora.nfw_terms(d1, d2 - h, R, c, inside)) / (2 * h)
        ref = np.array([fx[2], fy[2], fx[3], fy[3], fx[4], fy[4]])
        np.testing.assert_allclose(dt[:6], ref, rtol=1e-5, atol=1e-7 * np.abs(ref).max())
        fR = (ora.nfw_terms(d1, d2, R + h, c, inside) - ora.nfw_terms(d1, d2, R - h, c, inside)) / (2 * h)
        t = ora.nfw_terms(d1, d2, R, c, inside)
        if inside:
            np.testing.assert_allclose(dt[6:], fR[2:5], rtol=1e-5, atol=1e-7 * np.abs(fR[2:5]).max())
            np.testing.assert_allclose(t[5:7], fR[0:2], rtol=1e-5, atol=1e-7 * np.abs(fR[0:2]).max())
        else:
            assert np.all(dt[6:] == 0.0) and np.all(t[5:7] == 0.0)


def test_halo_tree_gradient_matches_frozen_finite_differences(ora):
    """L = sum ga . alpha + gk kappa + gg . gamma over a halo field: dL/d(m, x,
    y, R) of the frozen tree against finite differences."""
    lens, c = synth.nfw_halo_field(300, 141, rmax=0.3)
    rx, ry = synth.uniform_points(80, 142, -0.9, 0.9)
    g0 = synth.rng(143)
    ga, gk, gg = g0.normal(size=(rx.size, 2)), g0.normal(size=rx.size), g0.normal(size=(rx.size, 2))
    T = ora.Tree(lens.x, lens.y, lens.m, lens.s, c, 0.4, 4, 6, nfw=True)
    _, cnt = T.shoot(rx, ry, counts=True)
    assert cnt[:, 1].sum() > 0 and cnt[:, 4].sum() > 0
    dm, dx, dy, ds = T.grad(rx, ry, ga, gk=gk, gg=gg)
    T.record(rx, ry)
    base = {"x": lens.x, "y": lens.y, "m": lens.m, "s": lens.s}
    grads = {"x": dx, "y": dy, "m": dm, "s": ds}

    def loss(B):
        return float(np.sum(B[:, 0] * ga[:, 0] + B[:, 1] * ga[:, 1] + B[:, 2] * gk + B[:, 3] * gg[:, 0]
                            + B[:, 4] * gg[:, 1]))

    for i in synth.rng(144).choice(lens.n, 15, replace=False):
        for name in ["m", "x", "y", "s"]:
            h, vals = 1e-7, []
            for sgn in (1, -1):
                p = {k: v.copy() for k, v in base.items()}
                p[name][i] += sgn * h
                T.set_particles(p["x"], p["y"], p["m"], p["s"])
                vals.append(loss(T.shoot_frozen(rx, ry)))
            fd = (vals[0] - vals[1]) / (2 * h)
            gr = grads[name][i]
            assert abs(fd - gr) <= 1e-5 * max(abs(gr), 1e-3 * np.abs(grads[name]).max()), (name, i, fd, gr)
    T.set_particles(lens.x, lens.y, lens.m, lens.s)
