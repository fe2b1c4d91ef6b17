"""Writes the stored expected values under tests/golden/ from oracle/ only.

    python tests/golden/make_golden.py

oracle_a_point_masses_1k.txt: oracle A (FP64 brute force) at 64 seeded rays of
the 1,000-point-mass workload (m = 1e-3 in [-0.5, 0.5]^2, 64 x 64 ray grid).
Columns: ray index, x, y, alpha1, alpha2, kappa, gamma1, gamma2.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    oracle.build(force=False)
    lens, rx, ry = synth.workload_point_masses_1k()
    idx = synth.sample_rays(rx, ry, 64, synth.BASE_SEED + 100)
    A = oracle.direct(lens.x, lens.y, lens.m, lens.s, 3.0, rx[idx], ry[idx])
    rows = np.column_stack([idx, rx[idx], ry[idx], A])
    np.savetxt(os.path.join(HERE, "oracle_a_point_masses_1k.txt"), rows,
               fmt=["%d"] + ["%.17e"] * 7,
               header="ray x y alpha1 alpha2 kappa gamma1 gamma2 (oracle A, FP64)")


if __name__ == "__main__":
    main()
