"""Pins of oracle A (FP64 brute force) against what the paper and the
mathematics fix independently of the oracle's own formulas.

* kappa and gamma are defined as derivatives of alpha (Sec. 3.2): central finite
  differences of the oracle's alpha must reproduce its kappa and gamma, and the
  mixed derivatives must agree (alpha is a gradient).
* The surface density of a smoothed particle is the truncated Gaussian of
  Sec. 3.1: Gauss's law ties the flux of alpha through a circle to the
  enclosed mass, which the test integrates from the density by quadrature.
* A point mass has Einstein radius sqrt(m) in code units (Sec. 3.5): the
  magnification determinant built from the oracle's kappa and gamma vanishes
  there.
* Symmetry: a rotation by 90 degrees turns alpha as a vector and flips the
  sign of the spin-2 shear.
* Many particles in a uniform disk reproduce the analytic deflection of a
  uniform disk (Sec. 5.3: particle approximations of analytic profiles).
* n point masses on a circle: the closed form of the sum over the ring, and
  the exact multipole series of the same ring as one tree box.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import synth


def one(ora, x0, y0, m, s, q, rx, ry):
    return ora.direct(np.array([x0]), np.array([y0]), np.array([m]), np.array([s]), q,
                      np.asarray(rx, float), np.asarray(ry, float))


def fd_jacobian(ora, xs, ys, ms, ss, q, px, py, h):
    """Central differences of alpha at points (px, py): returns d alpha_i / d x_j."""
    px, py = np.asarray(px, float), np.asarray(py, float)
    ap = ora.direct(xs, ys, ms, ss, q, px + h, py)
    am = ora.direct(xs, ys, ms, ss, q, px - h, py)
    bp = ora.direct(xs, ys, ms, ss, q, px, py + h)
    bm = ora.direct(xs, ys, ms, ss, q, px, py - h)
    d1 = (ap - am) / (2 * h)  # d/dx1 of (a1, a2, ...)
    d2 = (bp - bm) / (2 * h)
    return d1, d2


@pytest.mark.parametrize("s", [0.0, 0.05, 0.2])
def test_kappa_gamma_are_derivatives_of_alpha(ora, s):
    g = synth.rng(101)
    q = 3.0
    xs = g.uniform(-0.3, 0.3, 5)
    ys = g.uniform(-0.3, 0.3, 5)
    ms = g.uniform(0.2, 1.0, 5)
    ss = np.full(5, s)
    px = g.uniform(-0.5, 0.5, 400)
    py = g.uniform(-0.5, 0.5, 400)
    # keep away from the support edge (kappa jumps there) and from the centres
    r = np.hypot(px[:, None] - xs[None], py[:, None] - ys[None])
    ok = np.all(np.abs(r - q * s) > 0.01, axis=1) & np.all(r > 0.02, axis=1)
    px, py = px[ok], py[ok]
    h = 1e-5
    d1, d2 = fd_jacobian(ora, xs, ys, ms, ss, q, px, py, h)
    out = ora.direct(xs, ys, ms, ss, q, px, py)
    scale = np.abs(d1[:, :2]).max(axis=1) + np.abs(d2[:, :2]).max(axis=1)
    kap = 0.5 * (d1[:, 0] + d2[:, 1])
    g1 = 0.5 * (d1[:, 0] - d2[:, 1])
    np.testing.assert_array_less(np.abs(kap - out[:, 2]) / scale, 1e-6)
    np.testing.assert_array_less(np.abs(g1 - out[:, 3]) / scale, 1e-6)
    np.testing.assert_array_less(np.abs(d2[:, 0] - out[:, 4]) / scale, 1e-6)
    np.testing.assert_array_less(np.abs(d1[:, 1] - out[:, 4]) / scale, 1e-6)  # curl free
    if s == 0.0:
        assert np.all(out[:, 2] == 0.0)


def test_gauss_law_matches_density_quadrature(ora):
    """Flux of alpha through circles = 2 x integral of kappa, where kappa is
    the truncated Gaussian density of Sec. 3.1 integrated independently."""
    q, s, m = 3.0, 0.1, 0.7
    C = -math.expm1(-q * q / 2)

    def density(r):  # Sigma / Sigma_crit in code units (m absorbs pi Sigma_crit)
        return m / (2 * s * s) * math.exp(-r * r / (2 * s * s)) / C if r < q * s else 0.0

    # an extra point mass outside every circle must add zero flux
    xs, ys = np.array([0.0, 0.9]), np.array([0.0, -0.4])
    ms, ss = np.array([m, 0.3]), np.array([s, 0.0])
    nphi = 2048
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    for R in [0.03, 0.1, 0.2, 0.29, 0.35, 0.5]:
        px, py = R * np.cos(ph), R * np.sin(ph)
        out = ora.direct(xs, ys, ms, ss, q, px, py)
        flux = np.sum(out[:, 0] * np.cos(ph) + out[:, 1] * np.sin(ph)) * R * 2 * math.pi / nphi
        enclosed, _ = integrate.quad(lambda r: 2 * math.pi * r * density(r), 0, R,
                                     points=[q * s] if R > q * s else None, limit=200)
        assert abs(flux - 2 * enclosed) < 1e-9 * max(1.0, 2 * enclosed), (R, flux, 2 * enclosed)


def test_total_convergence_is_pi_m(ora):
    """The integral of kappa over the plane is pi m in code units."""
    q, s, m = 3.0, 0.05, 0.37
    rr = np.linspace(0, q * s * (1 - 1e-13), 20001)
    out = one(ora, 0.0, 0.0, m, s, q, rr, np.zeros_like(rr))
    total = integrate.simpson(2 * math.pi * rr * out[:, 2], x=rr)
    assert abs(total - math.pi * m) < 1e-6


def test_point_lens_einstein_radius(ora):
    """det A = (1-kappa)^2 - |gamma|^2 vanishes at r_E = sqrt(m) (Sec. 3.5)."""
    for m in [1e-3, 0.25, 2.0]:
        def det(r):
            o = one(ora, 0.1, -0.2, m, 0.0, 3.0, [0.1 + r / math.sqrt(2)], [-0.2 + r / math.sqrt(2)])[0]
            return (1 - o[2]) ** 2 - o[3] ** 2 - o[4] ** 2

        rE = optimize.brentq(det, 0.1 * math.sqrt(m), 10 * math.sqrt(m), xtol=1e-15)
        assert abs(rE - math.sqrt(m)) < 1e-12 * math.sqrt(m)


def test_kernel_equals_point_mass_outside_support(ora):
    q, s, m = 3.0, 0.05, 0.8
    g = synth.rng(7)
    r = g.uniform(q * s * 1.0001, 1.0, 200)
    ph = g.uniform(0, 2 * math.pi, 200)
    px, py = r * np.cos(ph), r * np.sin(ph)
    a = one(ora, 0.0, 0.0, m, s, q, px, py)
    b = one(ora, 0.0, 0.0, m, 0.0, q, px, py)
    np.testing.assert_array_equal(a, b)
    # alpha is continuous across the support edge
    eps = 1e-9
    ain = one(ora, 0.0, 0.0, m, s, q, [q * s - eps], [0.0])[0]
    aout = one(ora, 0.0, 0.0, m, s, q, [q * s + eps], [0.0])[0]
    assert abs(ain[0] - aout[0]) < 1e-6 * abs(aout[0])


def test_kernel_centre_limits(ora):
    """Near the centre alpha -> kappa0 d, gamma -> 0, kappa -> kappa0 = m/(2 s^2 C)."""
    q, s, m = 3.0, 0.02, 1.0
    C = -math.expm1(-q * q / 2)
    k0 = m / (2 * s * s * C)
    d = np.array([1e-9, 1e-7, 1e-5])
    o = one(ora, 0.0, 0.0, m, s, q, d, np.zeros(3))
    np.testing.assert_allclose(o[:, 0], k0 * d, rtol=1e-6)
    np.testing.assert_allclose(o[:, 2], k0, rtol=1e-6)
    assert np.all(np.abs(o[:, 3]) < 1e-6 * k0)
    o0 = one(ora, 0.0, 0.0, m, s, q, [0.0], [0.0])[0]
    assert o0[0] == 0 and o0[1] == 0 and o0[3] == 0 and o0[4] == 0
    assert abs(o0[2] - k0) < 1e-12 * k0
    # a point mass exactly under a ray contributes nothing
    assert np.all(one(ora, 0.0, 0.0, m, 0.0, q, [0.0], [0.0]) == 0)


def test_rotation_and_reflection_covariance(ora):
    lens = synth.gaussian_blobs(200, 11, s_lo=0.02, s_hi=0.2)
    lens.m[::7] *= 3.0
    lens.s[::5] = 0.0
    px, py = synth.uniform_points(300, 12)
    a = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, px, py)
    # rotate everything by +90 degrees: (x, y) -> (-y, x)
    b = ora.direct(-lens.y, lens.x, lens.m, lens.s, lens.q, -py, px)
    sc = np.abs(a).max(axis=0)
    np.testing.assert_allclose(b[:, 0], -a[:, 1], atol=1e-12 * sc[0])
    np.testing.assert_allclose(b[:, 1], a[:, 0], atol=1e-12 * sc[0])
    np.testing.assert_allclose(b[:, 2], a[:, 2], atol=1e-12 * sc[2])
    np.testing.assert_allclose(b[:, 3:], -a[:, 3:], atol=1e-12 * sc[3])
    # reflect y -> -y
    c = ora.direct(lens.x, -lens.y, lens.m, lens.s, lens.q, px, -py)
    np.testing.assert_allclose(c[:, 0], a[:, 0], atol=1e-12 * sc[0])
    np.testing.assert_allclose(c[:, 1], -a[:, 1], atol=1e-12 * sc[0])
    np.testing.assert_allclose(c[:, 3], a[:, 3], atol=1e-12 * sc[3])
    np.testing.assert_allclose(c[:, 4], -a[:, 4], atol=1e-12 * sc[3])


def test_superposition_is_linear_in_mass(ora):
    lens = synth.gaussian_blobs(100, 21)
    px, py = synth.uniform_points(50, 22)
    a = ora.direct(lens.x, lens.y, lens.m, lens.s, lens.q, px, py)
    b = ora.direct(lens.x, lens.y, 2.5 * lens.m, lens.s, lens.q, px, py)
    np.testing.assert_allclose(b, 2.5 * a, rtol=1e-13, atol=1e-300)


def test_uniform_disk_from_particles(ora):
    """Smoothed particles filling a disk of radius R and mass M give
    alpha = M x / R^2 and kappa = M / R^2 well inside (Sec. 5.3, particle
    approximations of analytic lenses)."""
    n, R, M = 40000, 1.0, 1.0
    g = synth.rng(31)
    # Vogel's sunflower disk: a quiet, near-uniform particle layout
    i = np.arange(n)
    r = R * np.sqrt((i + 0.5) / n)
    ph = i * math.pi * (3 - math.sqrt(5))
    x, y = r * np.cos(ph), r * np.sin(ph)
    s = np.full(n, 0.04)
    m = np.full(n, M / n)
    pr = np.sqrt(g.uniform(0, 0.5 ** 2, 400))
    pph = g.uniform(0, 2 * math.pi, 400)
    px, py = pr * np.cos(pph), pr * np.sin(pph)
    out = ora.direct(x, y, m, s, 3.0, px, py)
    np.testing.assert_allclose(out[:, 2], M / R ** 2, rtol=2e-3)
    np.testing.assert_allclose(out[:, 0], M * px / R ** 2, atol=2e-3 * M / R)
    np.testing.assert_allclose(out[:, 1], M * py / R ** 2, atol=2e-3 * M / R)
    assert np.all(np.hypot(out[:, 3], out[:, 4]) < 2e-3 * M / R ** 2)
    # outside: a point mass M at the centre, to the same accuracy
    po = np.linspace(1.5, 3.0, 20)
    o2 = ora.direct(x, y, m, s, 3.0, po, np.zeros_like(po))
    np.testing.assert_allclose(o2[:, 0] * po / M, 1.0, atol=1e-4)


def test_kernel_norm(ora):
    assert abs(ora.kernel_norm(3.0) - (1 - math.exp(-4.5))) < 1e-15
    assert abs(ora.kernel_norm(1e-4) - (0.5e-8 - 0.125e-16)) < 1e-24


def test_point_mass_ring_closed_form(ora):
    """n equal point masses on a circle, z_j = b w^j (w = e^(2 pi i / n)): the
    sum over the ring has the closed form sum_j 1/(z - z_j) = n z^(n-1) / (z^n - b^n),
    so alpha1 - i alpha2 = m n z^(n-1) / (z^n - b^n) and, as its derivative,
    gamma1 - i gamma2 = -m n z^(n-2) (z^n + (n-1) b^n) / (z^n - b^n)^2 (the
    point lens of Sec. 3.5 superposed), inside and outside the ring."""
    n, m, a, phi0 = 7, 0.3, 0.4, 0.37
    b = a * np.exp(1j * phi0)
    zj = b * np.exp(2j * math.pi * np.arange(n) / n)
    g = synth.rng(131)
    r = np.concatenate([g.uniform(0.02, 0.3, 200), g.uniform(0.5, 3.0, 200)])
    ph = g.uniform(0, 2 * math.pi, 400)
    z = r * np.exp(1j * ph)
    assert np.min(np.abs(z[:, None] - zj[None])) > 0.05
    out = ora.direct(zj.real, zj.imag, np.full(n, m), np.zeros(n), 3.0, z.real, z.imag)
    F = m * n * z ** (n - 1) / (z ** n - b ** n)
    G = -m * n * z ** (n - 2) * (z ** n + (n - 1) * b ** n) / (z ** n - b ** n) ** 2
    scale = np.abs(F) + m / np.min(np.abs(z[:, None] - zj[None]), axis=1)
    assert np.all(np.abs((out[:, 0] - 1j * out[:, 1]) - F) <= 1e-13 * scale)
    gscale = np.abs(G) + m / np.min(np.abs(z[:, None] - zj[None]), axis=1) ** 2
    assert np.all(np.abs((out[:, 3] - 1j * out[:, 4]) - G) <= 1e-13 * gscale)
    assert np.all(out[:, 2] == 0.0)


def test_point_mass_ring_multipoles(ora):
    """The same ring as one accepted tree box: its moments about the centre are
    Q_k = n m b^k when n divides k and 0 otherwise, so the expansion to order p
    is exactly m n / z (1 + (b/z)^n [p >= n]) for alpha1 - i alpha2 and
    -m n / z^2 (1 + (n+1) (b/z)^n [p >= n]) for gamma1 - i gamma2 (Sec. 3.2,
    multipole expansion of a box)."""
    n, m, a, phi0 = 7, 0.3, 0.4, 0.37
    b = a * np.exp(1j * phi0)
    zj = b * np.exp(2j * math.pi * np.arange(n) / n)
    g = synth.rng(132)
    z = g.uniform(4.0, 8.0, 64) * np.exp(1j * g.uniform(0, 2 * math.pi, 64))
    for p in [0, 2, 6, 7, 9, 12]:
        T = ora.Tree(zj.real, zj.imag, np.full(n, m), np.zeros(n), 3.0, 0.9, n, p)
        assert T.ncells == 1
        B, cnt = T.shoot(z.real, z.imag, counts=True)
        assert np.all(cnt[:, 1] == 1)
        t = (b / z) ** n if p >= n else 0.0
        F = m * n / z * (1 + t)
        G = -m * n / z ** 2 * (1 + (n + 1) * t)
        assert np.all(np.abs((B[:, 0] - 1j * B[:, 1]) - F) <= 1e-14 * np.abs(F)), p
        assert np.all(np.abs((B[:, 3] - 1j * B[:, 4]) - G) <= 1e-14 * np.abs(G)), p
