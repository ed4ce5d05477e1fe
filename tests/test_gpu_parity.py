"""GPU parity of the HIP transport against the FP64 oracle (through the C ABI).

Deterministic (straight) mode: per-voxel relative agreement 1e-5 for voxels
above 1e-6 of the maximum, with an absolute floor of 1e-11 of the maximum.
Histories whose FP64 source position lies within 1e-4 mm of a voxel boundary
(or of the aperture edge) may land differently in FP32; their columns are
excluded and counted.

Full physics: independent seeds; >= 99 % of voxels above 10 % of the maximum
within 3 combined standard errors; mean dose over the high-dose region within
0.5 %; gamma 1 %/1 mm pass rate >= 99 %.
"""
import math
import sys

import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def gpu_q(eng, case, scen_index=0, physics=None, seed=None, k=None, grid_blocks=0, n_batches=0):
    eng.load_case(case)
    scen = [case.scenarios[scen_index]]
    dose, sig, led = eng.run_dose(case, 0, scenarios=scen, n_batches=n_batches, sigma=n_batches >= 2,
                                  physics=physics, seed=seed, fixed_point_bits=k or 0,
                                  grid_blocks=grid_blocks)
    q, kk = eng.last_tally(0)
    return q.cpu().numpy(), kk, dose[0].cpu().numpy(), (sig[0].cpu().numpy() if sig is not None else None), led[0]


def source_xy_fp64(orc, case, spot_index, n):
    """FP64 source positions of the first n histories of a spot (beam frame)."""
    f = case.fields[0]
    sp = f.spots[spot_index]
    key = [case.seed & 0xFFFFFFFF, ((case.seed >> 32) & 0xFFFFFFFF) ^ 0]
    xs = np.empty(n)
    ys = np.empty(n)
    for h in range(n):
        w = orc.philox([0, h, spot_index, 0], key)
        u0, u1 = orc.uniform(int(w[0])), orc.uniform(int(w[1]))
        r = math.sqrt(-2.0 * math.log(u0))
        xs[h] = float(sp["x_mm"]) + float(sp["sigma_mm"]) * r * math.cos(2 * math.pi * u1)
        ys[h] = float(sp["y_mm"]) + float(sp["sigma_mm"]) * r * math.sin(2 * math.pi * u1)
    return xs, ys


def edge_distance(poly, x, y):
    """Distance (mm) of BEV points (x, y) to the nearest polygon edge."""
    a = np.asarray(poly, np.float64)
    b = np.roll(a, -1, axis=0)
    d = np.full(x.shape, np.inf)
    for (ax_, ay_), (bx_, by_) in zip(a, b):
        ex, ey = bx_ - ax_, by_ - ay_
        t = np.clip(((x - ax_) * ex + (y - ay_) * ey) / (ex * ex + ey * ey), 0.0, 1.0)
        d = np.minimum(d, np.hypot(x - ax_ - t * ex, y - ay_ - t * ey))
    return d


def ambiguous_mask(orc, case, tol=1e-4, spots=None, shift_mm=(0.0, 0.0, 0.0)):
    """Voxels an FP32/FP64 rounding difference of the source position could
    change: the whole track line of every history that starts within tol of a
    lateral voxel boundary (or within 2e-3 mm of an aperture polygon edge or
    the range-shifter rim), and the neighbouring lines.  Beams must be
    axis-aligned.  spots: the spot indices of field 0 to cover (all by
    default); shift_mm: the scenario's isocentre shift (CT coordinates of a
    point move by -shift)."""
    g = case.geometry
    f = case.fields[0]
    nx, ny, nz = g.shape
    mask = np.zeros((nz, ny, nx), bool)
    ez = np.asarray(f.beam.ez)
    ax = int(np.argmax(np.abs(ez)))
    lat = [k for k in range(3) if k != ax]
    origin = np.asarray(g.origin, np.float64) + np.asarray(shift_mm, np.float64)
    for s in (range(len(f.spots)) if spots is None else spots):
        n = int(f.spots["n_histories"][s])
        x, y = source_xy_fp64(orc, case, s, n)
        p = np.asarray(f.beam.iso)[None, :] + x[:, None] * np.asarray(f.beam.ex)[None, :] \
            + y[:, None] * np.asarray(f.beam.ey)[None, :]
        fr = (p - origin[None, :]) / np.asarray(g.spacing)[None, :]
        bad = np.zeros(n, bool)
        for k in lat:
            bad |= np.abs(fr[:, k] - np.rint(fr[:, k])) * g.spacing[k] < tol
        r = np.hypot(x, y)
        if f.polygon is not None:
            bad |= edge_distance(f.polygon, x, y) < 2e-3
        if f.rs is not None:
            bad |= np.abs(r - 0.5 * f.rs.diameter_mm) < 2e-3
        for h in np.nonzero(bad)[0]:
            c = np.floor(fr[h]).astype(int)
            for d0 in (-1, 0, 1):
                for d1 in (-1, 0, 1):
                    idx = [slice(None)] * 3
                    i0, i1 = c[lat[0]] + d0, c[lat[1]] + d1
                    if not (0 <= i0 < g.shape[lat[0]] and 0 <= i1 < g.shape[lat[1]]):
                        continue
                    idx[2 - lat[0]] = i0
                    idx[2 - lat[1]] = i1
                    mask[tuple(idx)] = True
    return mask


def assert_straight_parity(q_gpu, k_gpu, q_or, k_or, excluded=None):
    a = q_gpu.astype(np.float64) * 2.0 ** -k_gpu
    b = q_or.astype(np.float64) * 2.0 ** -k_or
    dmax = b.max()
    assert dmax > 0
    keep = np.ones(b.shape, bool) if excluded is None else ~excluded
    hi = (b > 1e-6 * dmax) & keep
    rel = np.abs(a[hi] - b[hi]) / b[hi]
    lo = (~(b > 1e-6 * dmax)) & keep
    say(f"  straight parity: {hi.sum()} voxels, max rel {rel.max():.3e}, "
        f"excluded voxels {0 if excluded is None else int(excluded.sum())}")
    assert rel.max() <= 1e-5
    assert np.all(np.abs(a[lo] - b[lo]) <= 1e-11 * dmax)


# ------------------------------------------------------------- straight mode
def test_straight_parity_config1(eng, orc):
    c = I.config1(n_histories=100_000, physics=0)
    say("case config1 straight 1e5")
    qg, kg, dose, _, led = gpu_q(eng, c)
    qo, lo, ko = orc.run_tally(c)
    assert kg == ko
    assert_straight_parity(qg, kg, qo, ko, ambiguous_mask(orc, c))
    # dose conversion: FP32 dose equals the oracle conversion of the GPU tally
    ref = orc.q_to_gy(c, qg, kg)
    m = ref > 0
    np.testing.assert_allclose(dose[m], ref[m], rtol=2e-6)


@pytest.mark.parametrize("scale", [1.035, 0.965])
def test_straight_parity_range_scaled(eng, orc, scale):
    c = I.config1(n_histories=20_000, physics=0)
    c.scenarios = [I.Scenario(range_scale=scale)]
    say(f"case config1 straight range_scale={scale}")
    qg, kg, _, _, _ = gpu_q(eng, c)
    qo, _, ko = orc.run_tally(c)
    assert_straight_parity(qg, kg, qo, ko, ambiguous_mask(orc, c))


@pytest.mark.parametrize("opening,rs", [(10.0, True), (20.0, False), (40.0, True)])
def test_straight_parity_water_aperture(eng, orc, opening, rs):
    c = I.config2(opening, rs, histories_per_case=40_000, physics=0, shape=(64, 64, 200))
    say(f"case config2-small straight opening={opening} rs={rs} spots={len(c.fields[0].spots)}")
    qg, kg, _, _, lg = gpu_q(eng, c)
    qo, lo, ko = orc.run_tally(c)
    assert_straight_parity(qg, kg, qo, ko, ambiguous_mask(orc, c))
    e_or = lo * 2.0 ** -ko
    np.testing.assert_allclose(lg[1:3], e_or[1:3], rtol=1e-5, atol=1e-9 * e_or.sum())


@pytest.mark.parametrize("grid", [((128, 128, 80), (2.0, 2.0, 2.0)), ((256, 256, 320), (1.0, 1.0, 1.0))])
def test_straight_parity_head_ct(eng, orc, grid):
    """Head CT at 2 mm and at 1 mm (the resolution study's finest grid)."""
    g = I.head_ct(0, shape=grid[0], spacing=grid[1])
    c = I.config3(8.0, 400, physics=0, geometry=g, gantries=(90.0,))
    f = c.fields[0]
    f.spots = f.spots[:: max(1, len(f.spots) // 24)]
    say(f"case head straight grid={grid[1]} spots={len(f.spots)}")
    qg, kg, _, _, _ = gpu_q(eng, c)
    qo, _, ko = orc.run_tally(c)
    assert_straight_parity(qg, kg, qo, ko, ambiguous_mask(orc, c))


# ------------------------------------------------------------- determinism
def test_rerun_and_launch_shape_bitwise(eng):
    c = I.config2(20.0, True, histories_per_case=50_000, shape=(64, 64, 200))
    say("case rerun bitwise")
    q1, k1, d1, _, l1 = gpu_q(eng, c)
    q2, k2, d2, _, l2 = gpu_q(eng, c)
    q3, k3, d3, _, l3 = gpu_q(eng, c, grid_blocks=37)
    assert k1 == k2 == k3
    assert np.array_equal(q1, q2) and np.array_equal(q1, q3)
    assert np.array_equal(d1, d2) and np.array_equal(l1, l3)


def test_energy_balance_ledger(eng):
    c = I.config2(10.0, True, histories_per_case=20_000, shape=(64, 64, 200))
    say("case ledger balance")
    _, k, _, _, led = gpu_q(eng, c)
    f = c.fields[0]
    total = float(np.sum(f.spots["weight"].astype(np.float64) * f.spots["energy_mev"]))
    # ledger[0] is the grid; 1 RS, 2 block, 3 escaped, 4 nuclear
    n_dep = 400 * float(np.sum(f.spots["n_histories"]))
    assert led[:5].sum() == pytest.approx(total, abs=n_dep * 2.0 ** -k + 1e-6 * total)


# ------------------------------------------------------------- invariants
def test_wide_aperture_equals_no_aperture_bitwise_gpu(eng):
    g = I.water_geometry((60, 60, 120), (1.0, 1.0, 1.0))
    iso = (30.0, 30.0, 0.0)
    spots = I.make_spots([(0.0, 0.0)], 120.0, 3.0, 20_000)
    rs = I.RangeShifter(45.0, 61.0, 90.0)
    wide = I.Case("w", g, [I.Field(I.beam_along_z(iso), spots, I.circle_polygon(200.0, 256), I.Block(30, 8.5, 50), rs)],
                  [I.Scenario()])
    none = I.Case("n", g, [I.Field(I.beam_along_z(iso), spots, None, None, rs)], [I.Scenario()])
    say("case wide aperture")
    qa, ka, _, _, la = gpu_q(eng, wide, k=36)
    qb, kb, _, _, lb = gpu_q(eng, none, k=36)
    assert qa.any() and np.array_equal(qa, qb) and np.array_equal(la, lb)


def test_closed_aperture_zero_dose_gpu(eng):
    g = I.water_geometry((40, 40, 60), (1.0, 1.0, 1.0))
    spots = I.make_spots([(0.0, 0.0)], 147.0, 3.0, 20_000)
    c = I.Case("c", g, [I.Field(I.beam_along_z((20.0, 20.0, 0.0)), spots, None, I.Block(30, 8.5, 50), None)],
               [I.Scenario()])
    say("case closed aperture")
    q, k, d, _, led = gpu_q(eng, c)
    assert not q.any() and not d.any()
    assert led[2] + led[3] + led[4] == pytest.approx(147.0, rel=1e-5)


def test_lateral_shift_bitwise_gpu(eng):
    g = I.water_geometry((60, 40, 100), (1.0, 1.0, 1.0))
    g.origin = (64.0, 0.0, 0.0)
    spots = I.make_spots([(0.0, 0.0)], 100.0, 2.0, 20_000)
    sc = [I.Scenario(), I.Scenario(shift_mm=(3.0, 0.0, 0.0)), I.Scenario(shift_mm=(0.0, 0.0, 3.0))]
    c = I.Case("s", g, [I.Field(I.beam_along_z((94.0, 20.0, 0.0)), spots)], sc)
    say("case lateral shift")
    q0, k, _, _, _ = gpu_q(eng, c, 0, k=36)
    qx, _, _, _, _ = gpu_q(eng, c, 1, k=36)
    qz, _, _, _, _ = gpu_q(eng, c, 2, k=36)
    assert np.array_equal(qx[:, :, :-3], q0[:, :, 3:])
    assert np.array_equal(qz, q0)


# ------------------------------------------------------------- full physics
def stat_compare(orc, case, dg, sg, r, label):
    """3-sigma voxel test and the mean dose over the high-dose region (>= 50 %
    of the maximum of the two runs' mean); the
    mean-dose tolerance is 0.5 % or three standard errors of the difference
    when the runs are noisier than that (error of the oracle's regional mean
    from its batches, the same for the GPU run)."""
    do, so = r["dose_gy"], r["sigma_gy"]
    dmax = do.max()
    m = do >= 0.1 * dmax
    comb = np.sqrt(sg ** 2 + so ** 2)
    within = np.abs(dg - do) <= 3.0 * comb
    frac = within[m].mean()
    # the high-dose region is selected on the mean of the two doses: selecting
    # it on one side's own (noisy) dose biases that side's regional mean up
    avg = 0.5 * (dg + do)
    hi = avg >= 0.5 * avg.max()
    ratio = dg[hi].mean() / do[hi].mean()
    bm = np.array([b[hi].mean() for b in r["batch_dose_gy"]])
    se_rel = bm.std(ddof=1) / np.sqrt(len(bm)) / do[hi].mean()
    tol = max(0.005, 3.0 * np.sqrt(2.0) * se_rel)
    say(f"  {label}: 3-sigma fraction {frac:.4f} over {m.sum()} voxels; mean-dose ratio {ratio:.5f} "
        f"(tol {tol:.4f}, regional s.e. {se_rel:.4f}); U_gpu {np.mean(sg[hi] / dg[hi]):.4f} "
        f"U_or {np.mean(so[hi] / do[hi]):.4f}")
    assert frac >= 0.99
    assert abs(ratio - 1.0) <= tol
    return frac, ratio


def test_full_physics_config1_statistical(eng, orc):
    from gamma import gamma_pass_rate
    n = 2_000_000
    c = I.config1(n_histories=n, seed=0)
    say("case config1 full physics 2e6")
    _, _, dg, sg, _ = gpu_q(eng, c, n_batches=16)
    co = I.config1(n_histories=n, seed=12345)
    r = orc.dose(co, n_batches=16, keep_batches=True)
    stat_compare(orc, c, dg, sg, r, "config1")
    rate = gamma_pass_rate(r["dose_gy"], dg, c.geometry.spacing, 0.01, 1.0)
    say(f"  gamma 1%/1mm pass rate {rate:.4f}")
    assert rate >= 0.99
    # batch sigma of the GPU agrees with the oracle's
    hi = r["dose_gy"] >= 0.5 * r["dose_gy"].max()
    assert np.mean(sg[hi]) / np.mean(r["sigma_gy"][hi]) == pytest.approx(1.0, abs=0.1)


@pytest.mark.parametrize("opening,rs", [(10.0, True), (30.0, False)])
def test_full_physics_water_aperture_statistical(eng, orc, opening, rs):
    n = 3_000_000
    c = I.config2(opening, rs, histories_per_case=n, shape=(64, 64, 200), seed=0)
    say(f"case config2-small full physics opening={opening} rs={rs}")
    _, _, dg, sg, lg = gpu_q(eng, c, n_batches=16)
    co = I.config2(opening, rs, histories_per_case=n, shape=(64, 64, 200), seed=777)
    r = orc.dose(co, n_batches=16, keep_batches=True)
    stat_compare(orc, c, dg, sg, r, f"config2 {opening} {rs}")
    # energy balance agrees statistically (block and range shifter ledgers)
    e_or = r["ledger_mev"]
    np.testing.assert_allclose(lg[1:3], e_or[1:3], rtol=0.01, atol=1e-3 * e_or.sum())
