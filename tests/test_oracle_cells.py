"""Pins of the dynamic-voxel-spacing reference, no GPU: the identity
map returns the rows with the per-voxel dose; one cell per row gives the row
sum and the mass-weighted mean dose; merging never changes a row's total
energy; the run map of the inputs generator follows its structures."""
import numpy as np
import pytest

import oracle as O
from oracle import cells as OC
from paper_2307_01416_amd import inputs as I

MEVJ = 1.602176634e-13


def _rows(seed=0, n_rows=7, nvox=500):
    rng = np.random.default_rng(seed)
    cols, qs, ptr = [], [], [0]
    for _ in range(n_rows):
        c = np.sort(rng.choice(nvox, size=rng.integers(0, 60), replace=False))
        cols.append(c)
        qs.append(rng.integers(1, 1 << 40, size=c.size))
        ptr.append(ptr[-1] + c.size)
    return np.array(ptr), np.concatenate(cols).astype(np.int32), np.concatenate(qs).astype(np.int64)


def test_identity_map_keeps_the_rows():
    rp, col, q = _rows()
    mass = np.random.default_rng(1).uniform(0.5, 2.0, 500)
    p2, c2, q2, d2 = OC.cells_from_csr(rp, col, q, 30, np.arange(500), mass, 500, MEVJ)
    assert np.array_equal(p2, rp) and np.array_equal(c2, col) and np.array_equal(q2, q)
    np.testing.assert_allclose(d2, q * 2.0 ** -30 * MEVJ / (mass[col] * 1e-3), rtol=1e-15)


def test_one_cell_is_the_row_sum_and_the_mass_weighted_mean():
    rp, col, q = _rows(seed=2)
    mass = np.random.default_rng(3).uniform(0.5, 2.0, 500)
    p2, c2, q2, d2 = OC.cells_from_csr(rp, col, q, 30, np.zeros(500, np.int64), mass, 1, MEVJ)
    for r in range(len(rp) - 1):
        b, e = rp[r], rp[r + 1]
        if e == b:
            assert p2[r + 1] == p2[r]
            continue
        assert p2[r + 1] - p2[r] == 1
        assert q2[p2[r]] == q[b:e].sum()
        # dose = energy / mass: the mass-weighted mean of the voxel doses (zero where no entry)
        dv = np.zeros(500)
        dv[col[b:e]] = q[b:e] * 2.0 ** -30 * MEVJ / (mass[col[b:e]] * 1e-3)
        assert d2[p2[r]] == pytest.approx((dv * mass).sum() / mass.sum(), rel=1e-12)


def test_merging_keeps_every_row_total():
    rp, col, q = _rows(seed=4)
    cmap = np.repeat(np.arange(125), 4)
    p2, c2, q2, _ = OC.cells_from_csr(rp, col, q, 30, cmap, np.ones(500), 125, MEVJ)
    for r in range(len(rp) - 1):
        assert q2[p2[r]:p2[r + 1]].sum() == q[rp[r]:rp[r + 1]].sum()
        assert np.all(np.diff(c2[p2[r]:p2[r + 1]]) > 0)


def test_bad_maps_are_rejected():
    for m in (np.array([1, 1, 2]), np.array([0, 2, 2]), np.array([0, 1, 0])):
        with pytest.raises(ValueError):
            OC.check_map(m, int(m.max()) + 1)


def test_dynamic_spacing_map_follows_the_structures():
    shape = (20, 6, 4)
    roi = np.zeros(shape[::-1], np.uint8)
    roi[1, 2, 5:9] = 1          # target run: single voxels
    roi[2, 3, 0:10] = 2         # organ run: pairs
    cmap, n = I.dynamic_spacing_map(shape, roi.ravel(), target=1, oar=2, other=4)
    OC.check_map(cmap, n)
    c3 = cmap.reshape(shape[::-1])
    assert len(set(c3[1, 2, 5:9].tolist())) == 4
    assert len(set(c3[2, 3, 0:10].tolist())) == 5
    assert len(set(c3[0, 0, :].tolist())) == 5          # 20 voxels of tissue in runs of 4
    # runs never cross an x row
    assert len(set(c3[0, 0, :].tolist()) & set(c3[0, 1, :].tolist())) == 0
