"""The straight-mode parity bound (straight_bound.py) on the CPU, with the
oracle on both sides: moving every start by less than the rounding band is
absorbed by the per-history allowance; moving it by more, or changing one
voxel's tally by 2e-5, is caught."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import BAND_MM, allowance, assert_straight_parity


def _moved(case, dx):
    c = I.config2(10.0, True, histories_per_case=20_000, physics=0, shape=(64, 64, 200))
    f = c.fields[0]
    f.spots["x_mm"] = (f.spots["x_mm"].astype(np.float64) + dx).astype(np.float32)
    f.spots["y_mm"] = (f.spots["y_mm"].astype(np.float64) + 0.5 * dx).astype(np.float32)
    return c


@pytest.fixture(scope="module")
def base(orc):
    c = I.config2(10.0, True, histories_per_case=20_000, physics=0, shape=(64, 64, 200))
    q, _, k = orc.run_tally(c)
    allow, n = allowance(orc, c)
    return c, q, k, allow, n


def test_moves_within_the_band_are_covered(orc, base):
    c, q, k, allow, n = base
    assert n > 0
    # spot positions are FP32: the move actually applied is a few ulps of ~7 mm
    c2 = _moved(c, 0.4 * BAND_MM)
    q2, _, k2 = orc.run_tally(c2)
    assert k2 == k and not np.array_equal(q, q2)
    assert_straight_parity(q2, k2, q, k, allow)


def test_moves_beyond_the_band_fail(orc, base):
    c, q, k, allow, _ = base
    c2 = _moved(c, 2e-3)
    q2, _, k2 = orc.run_tally(c2)
    with pytest.raises(AssertionError):
        assert_straight_parity(q2, k2, q, k, allow)


def test_a_voxel_off_by_2e_5_fails(orc, base):
    c, q, k, allow, _ = base
    q2 = q.copy()
    b = q.astype(np.float64)
    v = np.unravel_index(np.argmax(np.where(allow == 0, b, 0.0)), q.shape)
    q2[v] += int(2e-5 * q[v]) + 1
    with pytest.raises(AssertionError):
        assert_straight_parity(q2, k, q, k, allow)
