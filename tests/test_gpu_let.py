"""Dose-averaged LET on the GPU against the FP64 oracle, through the
C ABI: each step's LET is its mean CSDA stopping power, the voxel's numerator
sum(dep * LET) is an int64 tally beside the dose tally.  Straight mode: the
numerator and LET_d per voxel to 1e-5 relative (voxels above 1e-6 of the
maximum dose, columns near voxel boundaries excluded as in the dose parity
tests); the dose tally is unchanged bit for bit by the LET tally.  Full
physics: depth profile of LET_d within 2 % where the dose is above 25 % of
its maximum, mean LET_d over the high-dose region within 1 %."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import allowance
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def gpu_let(eng, case, physics=None, seed=None, k=0):
    eng.load_case(case)
    eng.run_dose(case, 0, scenarios=[case.scenarios[0]], n_batches=0, sigma=False, physics=physics, seed=seed,
                 fixed_point_bits=k, let=True)
    q, kk = eng.last_tally(0)
    ql, sh = eng.last_let(0)
    return q.cpu().numpy(), ql.cpu().numpy(), kk, sh


def check_straight(orc, case, qg, qlg, kg, sh):
    qo, qlo, ko = orc.run_let(case)
    assert kg == ko and sh == orc.LET_SHIFT
    # a history starting within rounding of a boundary may deposit on the
    # other side of it: the oracle's allowances of the dose and of the LET
    # numerator (that history's start mirrored across the boundary) bound the
    # differences there; LET_d itself is compared where no such history deposits
    allow, _, allow_l = allowance(orc, case, with_let=True)
    keep = allow == 0
    b = qo.astype(np.float64)
    al_num = allow_l * 1.001 * 2.0 ** (ko - orc.LET_SHIFT) + np.where(allow_l > 0, 1e3, 0.0)
    num_err = np.abs(qlg.astype(np.float64) - qlo.astype(np.float64))
    assert np.all(num_err <= 1e-5 * qlo.astype(np.float64) + al_num + 1e-11 * qlo.max() + 2.0)
    al_q = allow * 1.001 * 2.0 ** ko + np.where(allow > 0, 1e3, 0.0)
    assert np.all(np.abs(qg.astype(np.float64) - b) <= 1e-5 * b + al_q + 1e-11 * b.max() + 1.0)
    hi = (b > 1e-6 * b.max()) & keep
    num_g, num_o = qlg.astype(np.float64)[hi], qlo.astype(np.float64)[hi]
    rel_num = np.abs(num_g - num_o) / np.maximum(num_o, 1.0)
    lg, lo = orc.let_d(qg, qlg)[hi], orc.let_d(qo, qlo)[hi]
    rel_let = np.abs(lg - lo) / lo
    say(f"  LET parity: {hi.sum()} voxels, numerator max rel {rel_num.max():.3e}, "
        f"LET_d max rel {rel_let.max():.3e}, LET_d range {lo.min():.3f}-{lo.max():.3f} keV/um")
    assert rel_num.max() <= 1e-5 and rel_let.max() <= 1e-5


def test_let_straight_config1(eng, orc):
    c = I.config1(n_histories=100_000, physics=0)
    say("case config1 straight 1e5 with LET")
    qg, qlg, kg, sh = gpu_let(eng, c)
    check_straight(orc, c, qg, qlg, kg, sh)
    # the dose tally does not depend on the LET tally
    eng.run_dose(c, 0, scenarios=[c.scenarios[0]], n_batches=0, sigma=False)
    q0, k0 = eng.last_tally(0)
    assert k0 == kg and np.array_equal(q0.cpu().numpy(), qg)


def test_let_straight_head_ct(eng, orc):
    g = I.head_ct(0, shape=(128, 128, 80), spacing=(2.0, 2.0, 2.0))
    c = I.config3(8.0, 400, physics=0, geometry=g, gantries=(90.0,))
    f = c.fields[0]
    f.spots = f.spots[:: max(1, len(f.spots) // 24)]
    say(f"case head straight spots={len(f.spots)} with LET")
    qg, qlg, kg, sh = gpu_let(eng, c)
    check_straight(orc, c, qg, qlg, kg, sh)


def test_let_full_physics_config1(eng, orc):
    n = 400_000
    c = I.config1(n_histories=n, seed=0)
    say("case config1 full physics 4e5 with LET")
    qg, qlg, kg, _ = gpu_let(eng, c)
    co = I.config1(n_histories=n, seed=4321)
    qo, qlo, ko = orc.run_let(co, threads=8)
    # depth profiles (lateral sums) of dose and numerator
    dg, ng = qg.sum(axis=(1, 2)).astype(np.float64), qlg.sum(axis=(1, 2)).astype(np.float64)
    do, no = qo.sum(axis=(1, 2)).astype(np.float64), qlo.sum(axis=(1, 2)).astype(np.float64)
    lg, lo = orc.let_d(dg, ng), orc.let_d(do, no)
    # slabs above a quarter of the peak dose (the distal fall-off, where LET_d
    # climbs steeply and few histories reach, is left to the mean below)
    m = do >= 0.25 * do.max()
    rel = np.abs(lg[m] - lo[m]) / lo[m]
    say(f"  LET_d depth profile: {m.sum()} slabs, max rel {rel.max():.3e}, "
        f"peak LET_d {lo[m].max():.3f} keV/um")
    assert rel.max() <= 0.02
    hi = qo >= 0.5 * qo.max()
    mg = orc.let_d(qg, qlg)[hi].mean()
    mo = orc.let_d(qo, qlo)[hi].mean()
    assert mg == pytest.approx(mo, rel=0.01)
