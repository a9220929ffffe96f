"""The seeded synthetic inputs: recipes are deterministic and have the stated
shapes and ranges (no GPU)."""
import math

import numpy as np

from paper_2010_11751_amd import workloads as W


def test_ensemble_recipe_is_seeded_and_in_range():
    e1 = W.ensemble(512)
    assert e1 == W.ensemble(512)
    assert min(m.n for m in e1) >= 16 and max(m.n for m in e1) <= 64
    assert all(100 <= m.re <= 1000 for m in e1)
    assert all(1.79 < m.omega < 1.995 for m in e1)
    cells = sum(m.n ** 3 for m in e1)
    assert 30e6 < cells < 60e6


def test_cavity_relaxation_frequencies():
    assert abs(W.CAVITY_SMALL.omega - 1.926040) < 1e-6
    assert abs(W.CAVITY_256.omega - 1.857355) < 1e-6
    assert abs(W.CAVITY_512.omega - 1.940391) < 1e-6
    assert W.CAVITY_256.fluid_cells == 16387064


def test_taylor_green_field_is_divergence_free_and_periodic():
    n = 16
    u = W.taylor_green_velocity(n, n, n, 0.04).reshape(3, n, n, n)
    div = sum((np.roll(u[a], -1, axis=a) - np.roll(u[a], 1, axis=a)) / 2 for a in range(3))
    k = 2 * math.pi / n
    assert np.abs(div).max() < 1e-15 + 0.04 * k ** 3
    assert abs(np.abs(u[0]).max() - 0.04) < 1e-12
