"""Pins of the lensing-potential oracle: alpha = grad psi and the Poisson
equation laplacian psi = 2 kappa (Sec. 3.2), the exponential-integral
function against scipy, continuity at the edge of the truncated support,
the point-mass closed form, and the tree's potential against the direct
sum."""
import numpy as np
import pytest

import synth


def test_ein_matches_scipy(ora):
    from scipy.special import exp1

    for z in (1e-8, 1e-3, 0.1, 0.5, 1.0, 2.0, 4.5, 8.0):
        ref = exp1(z) + np.euler_gamma + np.log(z)
        assert abs(ora.ein(z) - ref) <= 1e-14 * max(1.0, abs(ref)), z


@pytest.mark.parametrize("inside_r", [0.05, 0.7, 1.5, 2.9, 3.5, 6.0])
def test_gradient_and_laplacian_of_psi(ora, inside_r):
    s, q = 0.2, 3.0
    phi = 0.7
    d1, d2 = inside_r * s * np.cos(phi), inside_r * s * np.sin(phi)
    inside = inside_r < q

    def psi(a, b):
        return ora.unit_psi(a, b, s, q, ora_inside(a, b))

    def ora_inside(a, b):
        return a * a + b * b < (q * s) ** 2

    h = 1e-5 * s
    g1 = (psi(d1 + h, d2) - psi(d1 - h, d2)) / (2 * h)
    g2 = (psi(d1, d2 + h) - psi(d1, d2 - h)) / (2 * h)
    t = ora.unit_terms(d1, d2, s, q, inside)
    np.testing.assert_allclose([g1, g2], t[:2], rtol=1e-8, atol=1e-9 * np.hypot(*t[:2]))
    h = 1e-3 * s
    lap = (psi(d1 + h, d2) + psi(d1 - h, d2) + psi(d1, d2 + h) + psi(d1, d2 - h) - 4 * psi(d1, d2)) / (h * h)
    assert abs(lap - 2 * t[2]) <= 1e-5 * max(1.0, 2 * t[2] * s * s) / (s * s)


def test_continuity_and_point_mass(ora):
    s, q = 0.3, 3.0
    R = q * s
    inner = ora.unit_psi(R * (1 - 1e-12), 0.0, s, q, True)
    assert abs(inner - np.log(R)) < 1e-10
    assert ora.unit_psi(3.0, 4.0, 0.0, q, False) == np.log(5.0)
    # the centre value: ln R - Ein(q^2/2) / (2C)
    C = ora.kernel_norm(q)
    assert abs(ora.unit_psi(0.0, 0.0, s, q, True) - (np.log(R) - ora.ein(q * q / 2) / (2 * C))) < 1e-14


def test_direct_psi_gradient_is_direct_alpha(ora):
    lens = synth.gaussian_blobs(300, 91, s_lo=0.01, s_hi=0.2)
    lens.s[::5] = 0.0
    rx, ry = synth.uniform_points(40, 92)
    h = 1e-6
    p1 = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, 3.0, rx + h, ry)
    p0 = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, 3.0, rx - h, ry)
    q1 = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, 3.0, rx, ry + h)
    q0 = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, 3.0, rx, ry - h)
    ref = ora.direct(lens.x, lens.y, lens.m, lens.s, 3.0, rx, ry)
    np.testing.assert_allclose((p1 - p0) / (2 * h), ref[:, 0], rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose((q1 - q0) / (2 * h), ref[:, 1], rtol=1e-6, atol=1e-8)


def test_tree_psi(ora):
    lens = synth.gaussian_blobs(3000, 93, s_lo=0.003, s_hi=0.2)
    lens.s[::4] = 0.0
    rx, ry = synth.uniform_points(300, 94)
    ref = ora.direct_psi(lens.x, lens.y, lens.m, lens.s, 3.0, rx, ry)
    T0 = ora.Tree(lens.x, lens.y, lens.m, lens.s, 3.0, 0.0, 8, 2)
    np.testing.assert_allclose(T0.shoot_psi(rx, ry), ref, rtol=1e-12, atol=1e-13)
    errs = []
    for p in (2, 6, 10):
        T = ora.Tree(lens.x, lens.y, lens.m, lens.s, 3.0, 0.5, 8, p)
        errs.append(np.abs(T.shoot_psi(rx, ry) - ref).max() / np.abs(ref).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6, errs
