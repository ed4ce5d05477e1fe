"""The straight-mode parity bound (straight_bound.py) on the CPU, with the
oracle on both sides: moving every start by less than the rounding band is
absorbed by the per-history allowance; moving it by more, or changing one
voxel's tally by 2e-5, is caught."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import BAND_MM, allowance, assert_straight_parity, shift_allowance


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


def _div(dx=0.0):
    c = I.config2(20.0, True, histories_per_case=40_000, physics=0, shape=(64, 64, 200))
    f = c.fields[0]
    f.vsad_mm = 2000.0
    f.block = I.Block(f.block.thickness_mm, f.block.density_gcc, f.block.downstream_mm, focus_mm=2000.0)
    f.spots["x_mm"] = (f.spots["x_mm"].astype(np.float64) + dx).astype(np.float32)
    f.spots["y_mm"] = (f.spots["y_mm"].astype(np.float64) - 0.7 * dx).astype(np.float32)
    return c


@pytest.fixture(scope="module")
def div_base(orc):
    c = _div()
    q, _, k = orc.run_tally(c)
    return c, q, k, shift_allowance(orc, c)


def test_tilted_tracks_moved_within_the_band_are_covered(orc, div_base):
    """Virtual source and focused block: every history's crossings move when
    its start moves, and the shift allowance covers moves inside the band."""
    c, q, k, allow = div_base
    q2, _, k2 = orc.run_tally(_div(0.4 * BAND_MM))
    assert k2 == k and not np.array_equal(q, q2)
    assert_straight_parity(q2, k2, q, k, allow)


def test_tilted_tracks_moved_beyond_the_band_fail(orc, div_base):
    c, q, k, allow = div_base
    q2, _, k2 = orc.run_tally(_div(5e-3))
    with pytest.raises(AssertionError):
        assert_straight_parity(q2, k2, q, k, allow)


def test_move_allowance_of_a_history_that_does_not_move_is_zero(orc, div_base):
    """A zero move reproduces the history bit for bit (no allowance), and the
    traced move equals the difference of two single traces."""
    c = div_base[0]
    sp = c.fields[0].spots
    s = int(np.argmin(np.hypot(sp["x_mm"], sp["y_mm"])))     # a spot through the opening
    _, _, g0 = orc.trace_history(c, s, 17, want_grid=True)
    assert g0.any()
    assert not orc.move_allowance(c, [(s, 17, [(0.0, 0.0)])]).any()
    _, _, g1 = orc.trace_history(c, s, 17, want_grid=True, move=(0.3, -0.2))
    w = float(sp["weight"][s]) / float(sp["n_histories"][s])
    a = orc.move_allowance(c, [(s, 17, [(0.3, -0.2)])]).ravel()
    assert a.any()
    np.testing.assert_allclose(a, w * np.abs(g1 - g0), rtol=1e-12, atol=0)


def test_energy_moves_inside_the_direction_band_are_covered(orc, div_base):
    """A history of the virtual-source case whose energy moves by half the
    direction band's offset changes its deposits by no more than the
    allowance of the full +-offset moves, voxel by voxel."""
    from straight_bound import DIR_REL
    c = div_base[0]
    sp = c.fields[0].spots
    s = int(np.argmin(np.hypot(sp["x_mm"], sp["y_mm"])))
    e = float(sp["energy_mev"][s]) + 6.0 * float(sp["energy_sigma_mev"][s])
    de = DIR_REL * float(orc.csda_range(0, e)) * float(orc.stopping_power(0, e))
    w = float(sp["weight"][s]) / float(sp["n_histories"][s])
    checked = 0
    for h in range(40):
        _, _, g0 = orc.trace_history(c, s, h, want_grid=True)
        if not g0.any():
            continue
        a = orc.move_allowance(c, [(s, h, [(0.0, 0.0, de), (0.0, 0.0, -de)])]).ravel()
        for frac in (0.5, -0.3):
            _, _, g1 = orc.trace_history(c, s, h, want_grid=True, move=(0.0, 0.0, frac * de))
            assert np.all(w * np.abs(g1 - g0) <= a * (1 + 1e-9) + 1e-11 * w * g0)   # + FP64 rounding
        assert a.any()
        checked += 1
    assert checked >= 10
