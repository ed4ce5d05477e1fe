"""Divergent aperture block, virtual source and energy-layer-specific
apertures (the paper's next steps in its Discussion) on the GPU
against the FP64 oracle, through the C ABI.

Workload: config 2 geometry (water, 30 mm brass block 50 mm upstream of the
surface, 20 mm circular opening, 45 mm WET range shifter) with the beam
diverging from a virtual source 2 m upstream and the block's walls focused
on it (and the block alone focused, beam parallel; and the beam alone
divergent, block walls parallel).

Straight mode: the straight-mode bar of the other tests, 1e-5 per voxel
above 1e-6 of the maximum plus a per-voxel allowance, here for every history:
a tilted track's crossings of lateral voxel boundaries and of tilted walls
move along it by (start error) / tilt, so each history is transported by the
oracle with its start moved by the FP32 rounding band along the eight
directions of the source plane's square, and the largest change of its
deposits in each voxel is its allowance there (straight_bound.shift_allowance;
the allowances add up to at most 0.2 % of the dose).  Depth slices (sums over
the lateral plane, which such moves do not change) are held to 2e-5, the
block and range-shifter ledgers to 1e-4.  Full physics: the bar of the other
physics parity tests (3 sigma on >= 99 % of the voxels above 10 %, mean dose
over the high-dose region within a fixed 0.5 %, gamma 1 %/1 mm on >= 99 %)."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import assert_straight_parity, shift_allowance
from test_gpu_parity import gpu_q, say, stat_compare_oracle, straight_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def div_case(n, physics, seed=0, vsad=2000.0, focus=2000.0, rs=True, opening=20.0):
    c = I.config2(opening, rs, histories_per_case=n, shape=(64, 64, 200), seed=seed, physics=physics)
    f = c.fields[0]
    f.vsad_mm = vsad
    f.block = I.Block(f.block.thickness_mm, f.block.density_gcc, f.block.downstream_mm, focus_mm=focus)
    c.name = f"config2_div_{int(opening)}_{vsad:.0f}_{focus:.0f}"
    return c


@pytest.mark.parametrize("vsad,focus", [(2000.0, 2000.0), (0.0, 2000.0), (2000.0, 0.0)])
def test_straight_parity_divergent(eng, orc, vsad, focus):
    c = div_case(200_000, 0, vsad=vsad, focus=focus)
    say(f"case {c.name} straight")
    qg, kg, _, _, lg = gpu_q(eng, c)
    qo, led_o, ko = orc.run_tally(c)
    assert_straight_parity(qg, kg, qo, ko, shift_allowance(orc, c), say=say)
    a = qg.astype(np.float64) * 2.0 ** -kg
    b = qo.astype(np.float64) * 2.0 ** -ko
    sa = a.reshape(200, -1).sum(1)
    sb = b.reshape(200, -1).sum(1)
    m = sb > 1e-3 * sb.max()
    srel = np.abs(sa[m] - sb[m]) / sb[m]
    lo = led_o.astype(np.float64) * 2.0 ** -ko
    lrel = np.abs(np.asarray(lg[1:3]) - lo[1:3]) / np.maximum(lo[1:3], 1e-300)
    say(f"  slices max rel {srel.max():.2e}; RS/block ledgers rel {lrel}")
    assert srel.max() <= 2e-5
    assert np.all(lrel <= 1e-4)


@pytest.mark.parametrize("vsad,focus", [(2000.0, 2000.0), (2000.0, 0.0)])
def test_full_physics_divergent_statistical(eng, orc, vsad, focus):
    n = 4_000_000
    c = div_case(4 * n, I.PHYS_ALL, vsad=vsad, focus=focus)
    say(f"case {c.name} full physics: oracle 4e6, GPU 1.6e7")
    _, _, dg, sg, lg = gpu_q(eng, c, n_batches=16)
    co = div_case(n, I.PHYS_ALL, seed=777, vsad=vsad, focus=focus)
    r = orc.dose(co, n_batches=16, keep_batches=True)
    stat_compare_oracle(dg, sg, r, c, c.name)
    e_or = r["ledger_mev"]
    np.testing.assert_allclose(lg[1:3], e_or[1:3], rtol=0.01, atol=1e-3 * e_or.sum())


def test_far_focus_and_far_source_match_the_parallel_geometry(eng):
    """A focus and a virtual source 1e9 mm away give the non-divergent,
    parallel-beam dose (rays tilt by < 3e-8 rad)."""
    a = gpu_q(eng, div_case(100_000, 0, vsad=0.0, focus=0.0))
    b = gpu_q(eng, div_case(100_000, 0, vsad=1e9, focus=1e9))
    qa = a[0].astype(np.float64) * 2.0 ** -a[1]
    qb = b[0].astype(np.float64) * 2.0 ** -b[1]
    assert np.abs(qa - qb).sum() <= 1e-5 * qa.sum()


def test_straight_parity_layer_aperture_head_ct(eng, orc):
    """Energy-layer-specific apertures (one field per energy layer, opening =
    the target's cross-section at the layer's depth + 5 mm): straight-mode
    parity on the head CT for the layer with the smallest opening and for a
    central one."""
    g = I.head_ct(0, shape=(128, 128, 80), spacing=(2.0, 2.0, 2.0))
    c = I.config3(8.0, 400, physics=0, geometry=g, gantries=(90.0,), layer_apertures=True, n_vertices=32)
    radii = [float(np.abs(f.polygon).max()) for f in c.fields]
    for fi in (int(np.argmin(radii)), int(np.argmax(radii))):
        sub = I.Case(f"layer{fi}", g, [c.fields[fi]], c.scenarios, physics=0)
        f = sub.fields[0]
        f.spots = f.spots[:: max(1, len(f.spots) // 24)]
        say(f"case head layer aperture field {fi} radius {radii[fi]:.1f} spots={len(f.spots)}")
        qg, kg, _, _, _ = gpu_q(eng, sub)
        qo, _, ko = orc.run_tally(sub)
        straight_check(orc, sub, qg, kg, qo, ko)


@pytest.mark.parametrize("physics", [0, I.PHYS_ALL])
def test_divergent_csr_rows_sum_to_dense(eng, physics):
    """The work-queue influence-matrix path with a divergent field (its
    divergent specialisation): the rows sum to the dense tally bit for bit,
    and the same holds on the plain specialisation for the plain field."""
    for vsad, focus in ((2000.0, 2000.0), (0.0, 0.0)):
        c = div_case(60_000, physics, vsad=vsad, focus=focus)
        say(f"case {c.name} csr vs dense physics={physics}")
        rp, col, val, q, k = eng.run_csr(c, fixed_point_bits=36)
        eng.load_case(c)
        eng.run_dose(c, sigma=False, fixed_point_bits=36)
        qd, kd = eng.last_tally(0)
        dense = np.zeros(c.geometry.nvox, np.int64)
        np.add.at(dense, col, q)
        assert np.array_equal(dense, qd.cpu().numpy().ravel())
