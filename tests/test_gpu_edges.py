"""Edge cases of the transport on the GPU against the FP64 oracle, through
the C ABI, in straight mode (no random numbers after the source, so the
per-voxel bar is the deterministic one: 1e-5 relative plus the start-rounding
allowance of straight_bound.py):

* ragged history counts (1, 63, 64, 65, 127, 129 and 1000 VPs per spot,
  against work chunks of 64 x histories-per-lane), dense and as influence
  rows;
* spots with no histories and spots that miss the grid: empty rows, no dose,
  their energy in the escaped ledger;
* energies at the ends of the tables (3 MeV stops inside the first voxel,
  250 MeV leaves the grid);
* degenerate grids: a single voxel, a 3 x 2 x 1 slab and a one-voxel-wide
  column.

Ledgers (MeV x w/N, fixed point) match the oracle's to 1e-6 of the energy
put in, and grid + escaped + range-shifter + block ledgers add up to it."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import allowance, assert_straight_parity
from test_gpu_parity import gpu_q, say, straight_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def pencil_case(name, shape, spacing, spots, physics=0):
    g = I.water_geometry(shape, spacing)
    nx, ny, _ = g.shape
    iso = (0.5 * nx * g.spacing[0], 0.5 * ny * g.spacing[1], 0.0)
    f = I.Field(beam=I.beam_along_z(iso), spots=spots)
    return I.Case(name, g, [f], [I.Scenario()], physics=physics)


def spot_table(rows):
    """rows: (x, y, energy, sigma, n_histories)"""
    s = np.zeros(len(rows), dtype=I.SPOT_DTYPE)
    for i, (x, y, e, sg, n) in enumerate(rows):
        s[i]["x_mm"], s[i]["y_mm"], s[i]["energy_mev"], s[i]["sigma_mm"] = x, y, e, sg
        s[i]["energy_sigma_mev"] = 0.0
        s[i]["weight"] = 1.0
        s[i]["n_histories"] = n
    return s


def energy_in(case):
    sp = case.fields[0].spots
    return float(np.sum(sp["weight"].astype(np.float64) * (sp["n_histories"] > 0) * sp["energy_mev"]))


def check_dense(eng, orc, case):
    """Straight parity of the dense tally with the start allowance, and the
    ledgers: equal to the oracle's within 1e-6 of the energy put in plus the
    whole energy of each history whose start may round across a boundary
    (on a one-voxel grid that can decide between hitting and missing it)."""
    qg, kg, _, _, lg = gpu_q(eng, case)
    qo, led_o, ko = orc.run_tally(case)
    assert kg == ko
    allow, n_amb = allowance(orc, case)
    say(f"  {n_amb} histories start within rounding of a boundary")
    assert_straight_parity(qg, kg, qo, ko, allow, say=say)
    lo = led_o.astype(np.float64) * 2.0 ** -ko
    e_in = energy_in(case)
    sp = case.fields[0].spots
    n = np.maximum(sp["n_histories"].astype(np.float64), 1.0)
    per_hist = float(np.max(sp["weight"].astype(np.float64) * sp["energy_mev"] / n))
    tol = 1e-6 * e_in + n_amb * per_hist
    say(f"  ledgers gpu {np.round(lg, 6)} oracle {np.round(lo, 6)} energy in {e_in:.6f}")
    np.testing.assert_allclose(np.asarray(lg, np.float64), lo, rtol=0, atol=tol)
    assert abs(float(np.sum(lo)) - e_in) <= 1e-6 * e_in
    assert abs(float(np.sum(lg)) - e_in) <= 1e-6 * e_in
    return qg, kg


def test_ragged_history_counts_dense_and_rows(eng, orc):
    counts = [1, 63, 64, 65, 127, 129, 1000]
    rows = [(-12.0 + 4.0 * i, 1.5 * (i % 3) - 1.5, 100.0, 3.0, n) for i, n in enumerate(counts)]
    c = pencil_case("ragged", (40, 40, 80), (2.0, 2.0, 2.0), spot_table(rows))
    say(f"case ragged history counts {counts}")
    qg, kg = check_dense(eng, orc, c)
    ref = orc.spot_tallies(c, k=kg)
    for hpl in (1, 2, 3):
        rp, col, _, q, k = eng.run_csr(c, fixed_point_bits=kg, hist_per_lane=hpl)
        assert k == kg
        dense = np.zeros(c.geometry.nvox, np.int64)
        np.add.at(dense, col, q)
        assert np.array_equal(dense, qg.ravel()), f"rows at {hpl} histories per lane"
        if hpl != 2:
            continue
        # every row against the oracle's tally of its spot alone
        for s, r in enumerate(ref):
            a, b = int(rp[s]), int(rp[s + 1])
            row = np.zeros(c.geometry.nvox, np.int64)
            row[col[a:b]] = q[a:b]
            assert b > a
            straight_check(orc, c, row.reshape(qg.shape), k, r, k, spots=[s])


def test_empty_and_missing_spots(eng, orc):
    rows = [(0.0, 0.0, 120.0, 3.0, 500),        # an ordinary spot
            (2.0, 0.0, 120.0, 3.0, 0),          # no histories
            (500.0, 0.0, 120.0, 3.0, 300),      # misses the grid
            (0.0, -3.0, 90.0, 3.0, 400)]
    c = pencil_case("empty_missing", (40, 40, 80), (2.0, 2.0, 2.0), spot_table(rows))
    say("case spots with no histories and a spot that misses the grid")
    qg, kg = check_dense(eng, orc, c)
    rp, col, _, q, k = eng.run_csr(c, fixed_point_bits=kg)
    nnz = np.diff(rp)
    say(f"  row entries {nnz.tolist()}")
    assert nnz[1] == 0 and nnz[2] == 0 and nnz[0] > 0 and nnz[3] > 0
    dense = np.zeros(c.geometry.nvox, np.int64)
    np.add.at(dense, col, q)
    assert np.array_equal(dense, qg.ravel())


@pytest.mark.parametrize("energy", [3.0, 250.0])
def test_table_end_energies(eng, orc, energy):
    rows = [(0.0, 0.0, energy, 2.0, 3000)]
    c = pencil_case(f"energy_{energy:g}", (30, 30, 80), (2.0, 2.0, 2.0), spot_table(rows))
    say(f"case {energy} MeV pencil beam")
    qg, kg = check_dense(eng, orc, c)
    depth = qg.reshape(80, -1).sum(1)
    if energy < 10.0:
        assert depth[0] > 0 and depth[1:].sum() == 0   # range ~0.2 mm
    else:
        assert depth[-1] > 0                         # leaves through the far face


@pytest.mark.parametrize("shape,spacing", [((1, 1, 1), (2.0, 2.0, 2.0)), ((3, 2, 1), (1.0, 1.0, 3.0)),
                                           ((1, 1, 200), (1.0, 1.0, 1.0))])
def test_degenerate_grids(eng, orc, shape, spacing):
    rows = [(0.0, 0.0, 60.0, 0.3, 2000), (0.2, -0.1, 30.0, 0.2, 700)]
    c = pencil_case(f"grid_{shape}", shape, spacing, spot_table(rows))
    say(f"case grid {shape} at {spacing} mm")
    qg, kg = check_dense(eng, orc, c)
    assert qg.sum() > 0
    rp, col, _, q, k = eng.run_csr(c, fixed_point_bits=kg)
    dense = np.zeros(c.geometry.nvox, np.int64)
    np.add.at(dense, col, q)
    assert np.array_equal(dense, qg.ravel())
