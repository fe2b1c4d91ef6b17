"""Stored oracle values (written by tests/golden/make_golden.py from oracle/
only) and closed-form values from the paper."""
import math
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_oracle_a_reproduces_stored_values(ora):
    rows = np.loadtxt(os.path.join(GOLDEN, "oracle_a_point_masses_1k.txt"))
    lens, rx, ry = synth.workload_point_masses_1k()
    idx = rows[:, 0].astype(int)
    np.testing.assert_array_equal(rx[idx], rows[:, 1])
    A = ora.direct(lens.x, lens.y, lens.m, lens.s, 3.0, rx[idx], ry[idx])
    np.testing.assert_allclose(A, rows[:, 3:], rtol=1e-13, atol=1e-15)


def test_point_lens_closed_form_values(ora):
    """Sec. 3.5: alpha = r_E^2 / r, so for m = 1e-3 the Einstein radius is
    0.0316227766 and a ray at r_E is deflected by exactly r_E."""
    rE = math.sqrt(1e-3)
    A = ora.direct(np.zeros(1), np.zeros(1), np.array([1e-3]), np.zeros(1), 3.0,
                   np.array([rE]), np.array([0.0]))[0]
    assert abs(A[0] - 0.031622776601683794) < 1e-16
    assert A[1] == 0 and A[2] == 0
    assert abs(A[3] + 1.0) < 1e-15  # |gamma| = 1 at the Einstein radius
