"""The stored oracle trajectory of the 16^3 cube is a discharge (CPU).

tests/golden/cube16_q1_trajectory.npz holds the oracle's steady initial
state and the roots of five backward-Euler steps of 0.1 s at 0.1C (written
by tests/golden/make_cube16_trajectory.py from the oracle alone).  Before
the GPU trajectory is compared with it, check that the file is what it
claims: successive step roots of a galvanostatic discharge, whose lithium
count rises by the separator inflow j_el A dt / F per step, whose sulfur
count is kept, and whose reaction current carries j_el A (the conservation
statements of Sec. 3.2 for the discrete scheme).
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube16_q1_trajectory.npz")


def test_oracle_trajectory_is_a_discharge():
    if not os.path.exists(GOLDEN):
        pytest.fail(f"missing {GOLDEN} (python tests/golden/make_cube16_trajectory.py)")
    with np.load(GOLDEN, allow_pickle=False) as z:
        s, t, j_el, dt, u = z["sums"], z["t"], float(z["j_el"]), float(z["dt"]), z["u"]
    assert u.shape == (6, 9, 4096, 8)
    assert np.allclose(np.diff(t), dt)
    area = 16 * 16 * 1e-12
    q = dt * j_el * area / 96485.332
    assert np.all(np.abs(np.diff(s[:, 0])) < 1e-12 * s[0, 0])
    assert np.all(np.abs(np.diff(s[:, 1]) - q) < 1e-12 * s[0, 1])
    assert np.all(np.abs(s[:, 3] / (j_el * area) - 1.0) < 1e-8)
    assert np.all(u[1:, 0:6] > 0)
