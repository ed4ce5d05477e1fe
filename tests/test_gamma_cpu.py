"""Pins of the gamma tool on analytic cases and against a brute-force
evaluation of the same definition."""
import math

import numpy as np
import pytest
from scipy import special

from gamma import gamma_bruteforce, gamma_pass_rate


def test_identical_is_100_percent():
    rng = np.random.default_rng(0)
    a = rng.uniform(0.5, 1.0, size=(6, 7, 8))
    assert gamma_pass_rate(a, a, (1, 1, 1), 0.01, 1.0) == 1.0


def test_uniform_scaling_flat_region():
    a = np.ones((5, 6, 7))
    assert gamma_pass_rate(a, 1.009 * a, (1, 1, 1), 0.01, 1.0) == 1.0
    assert gamma_pass_rate(a, 1.011 * a, (1, 1, 1), 0.01, 1.0) == 0.0


def test_shifted_steep_edge_passes_within_dta():
    # lateral penumbra (erfc edge, width 1.5 mm) on 0.5 mm voxels
    x = (np.arange(60) + 0.5) * 0.5
    def edge(c):
        return np.broadcast_to(0.5 * special.erfc((x - c) / 1.5), (3, 3, 60)).copy()
    ref = edge(15.0)
    # an offset on the search sub-grid, and 0.8 mm with a finer sub-grid
    assert gamma_pass_rate(ref, edge(15.75), (0.5, 0.5, 0.5), 0.01, 1.0) == 1.0
    assert gamma_pass_rate(ref, edge(15.8), (0.5, 0.5, 0.5), 0.01, 1.0, substep=0.05) == 1.0
    assert gamma_pass_rate(ref, edge(16.5), (0.5, 0.5, 0.5), 0.01, 1.0) < 0.9


def test_matches_bruteforce_on_tiny_grids():
    rng = np.random.default_rng(3)
    for _ in range(3):
        ref = rng.uniform(0.0, 1.0, size=(4, 4, 5))
        ev = ref * rng.uniform(0.97, 1.03, size=ref.shape)
        sp = (1.0, 1.5, 2.0)
        a = gamma_pass_rate(ref, ev, sp, 0.02, 1.0)
        b = gamma_bruteforce(ref, ev, sp, 0.02, 1.0)
        assert a == pytest.approx(b, abs=1e-12)
