"""GPU checks of the influence-matrix (CSR) builder and the batched
work-queue pass: every row equals the oracle's per-spot tally (straight
mode, same voxels and values to 1e-5; full physics bitwise against the GPU's
own dense single-spot runs), columns ascend, the rows of a scenario sum to
its dense tally bitwise, reruns are bit-identical."""
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


def rows_of(row_ptr, col, q):
    out = []
    for r in range(len(row_ptr) - 1):
        a, b = int(row_ptr[r]), int(row_ptr[r + 1])
        out.append((col[a:b], q[a:b]))
    return out


def small_case(physics, n=3000, opening=20.0, rs=True):
    c = I.config2(opening, rs, histories_per_case=n * 10, physics=physics, shape=(48, 48, 160))
    c.fields[0].spots = c.fields[0].spots[:: max(1, len(c.fields[0].spots) // 10)]
    c.fields[0].spots["n_histories"] = n
    return c


def test_csr_rows_equal_oracle_straight(eng, orc):
    c = small_case(0)
    say(f"case csr straight spots={len(c.fields[0].spots)}")
    rp, col, val, q, k = eng.run_csr(c, fixed_point_bits=36)
    rows = rows_of(rp, col, q)
    for s, (cc, qq) in enumerate(rows):
        qo, _, _ = orc.run_tally(c, k=36, spots=(s, s + 1))
        qo = qo.ravel()
        nz = np.nonzero(qo)[0]
        assert np.all(np.diff(cc) > 0)
        # same support except voxels whose oracle value is tiny
        big = nz[qo[nz] > 1e-6 * qo.max()]
        assert np.isin(big, cc).all()
        ref = qo[cc].astype(np.float64)
        m = ref > 1e-6 * qo.max()
        rel = np.abs(qq[m] - ref[m]) / ref[m]
        assert rel.max() <= 2e-5, (s, rel.max())


def test_csr_rows_sum_to_dense_and_rerun_bitwise(eng):
    c = small_case(I.PHYS_ALL)
    say("case csr vs dense bitwise")
    rp, col, val, q, k = eng.run_csr(c, fixed_point_bits=36)
    rp2, col2, val2, q2, _ = eng.run_csr(c, fixed_point_bits=36, hist_per_lane=1, max_slots=3)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2) and np.array_equal(q, q2)
    eng.load_case(c)
    eng.run_dose(c, sigma=False, fixed_point_bits=36)
    qd, kd = eng.last_tally(0)
    dense = np.zeros(c.geometry.nvox, np.int64)
    np.add.at(dense, col, q)
    assert np.array_equal(dense, qd.cpu().numpy().ravel())
    # values are the FP32 conversion of the int64 tallies
    assert np.all(val > 0) and np.all(np.isfinite(val))


def test_batched_rows_equal_single_spot_dense_runs(eng):
    c = small_case(I.PHYS_ALL, n=2000)
    c.scenarios = I.scenarios_13()[:3]
    say("case batched vs single-spot dense")
    rp, col, val, q, k = eng.run_csr(c, fixed_point_bits=36)
    rows = rows_of(rp, col, q)
    n_sp = len(c.fields[0].spots)
    assert len(rows) == 3 * n_sp
    eng.load_case(c)
    for sc in range(3):
        for s in (0, n_sp - 1):
            one = I.Case("one", c.geometry, [c.fields[0]], [c.scenarios[sc]], seed=c.seed, physics=c.physics)
            w = c.fields[0].spots["weight"].copy()
            saved = c.fields[0].spots.copy()
            c.fields[0].spots["weight"] = 0.0
            c.fields[0].spots["weight"][s] = w[s]
            eng.run_dose(one, sigma=False, fixed_point_bits=36)
            c.fields[0].spots = saved
            qd, _ = eng.last_tally(0)
            qd = qd.cpu().numpy().ravel()
            cc, qq = rows[sc * n_sp + s]
            assert np.array_equal(np.nonzero(qd)[0], cc)
            assert np.array_equal(qd[cc], qq)


def test_graph_capture_equals_eager(eng):
    """The whole multi-epoch pass captured in one hipGraph gives the eager
    rows bit for bit, also when its first capacity is too small (the graph
    reports the overflow and the eager path reruns)."""
    c = small_case(I.PHYS_ALL, n=4000)
    c.scenarios = I.scenarios_13()[:2]
    say("case csr graph vs eager")
    rp, col, _, q, _ = eng.run_csr(c, fixed_point_bits=36, max_slots=4)
    rpg, colg, _, qg, _ = eng.run_csr(c, fixed_point_bits=36, max_slots=4, graph=True)
    assert np.array_equal(rp, rpg) and np.array_equal(col, colg) and np.array_equal(q, qg)
    big = small_case(I.PHYS_ALL, n=40000)
    big.scenarios = I.scenarios_13()[:2]
    rp2, col2, _, q2, _ = eng.run_csr(big, fixed_point_bits=36, max_slots=4, graph=True)
    rp3, col3, _, q3, _ = eng.run_csr(big, fixed_point_bits=36, max_slots=4)
    assert rp2[-1] > rp[-1]
    assert np.array_equal(rp2, rp3) and np.array_equal(col2, col3) and np.array_equal(q2, q3)


def test_head_three_fields_rows_sum_to_dense(eng):
    """Synthetic head, three fields with their own apertures and range
    shifters, two scenarios, one work queue: per scenario, the rows of all
    fields sum to the sum of the three fields' dense tallies, bit for bit."""
    g = I.head_ct(0, shape=(128, 128, 80), spacing=(2.0, 2.0, 2.0))
    c = I.config3(8.0, 300, geometry=g)
    for f in c.fields:
        f.spots = f.spots[:: max(1, len(f.spots) // 12)].copy()
    c.scenarios = [I.Scenario(), I.Scenario(shift_mm=(0.0, 3.0, 0.0), range_scale=0.965)]
    say(f"case head 3 fields csr: spots {[len(f.spots) for f in c.fields]}")
    rp, col, _, q, _ = eng.run_csr(c, fixed_point_bits=34)
    rows = rows_of(rp, col, q)
    n_per_scen = sum(len(f.spots) for f in c.fields)
    assert len(rows) == 2 * n_per_scen
    eng.load_case(c)
    for sc in range(2):
        dense = np.zeros(g.nvox, np.int64)
        for fi in range(3):
            eng.run_dose(c, fi, scenarios=[c.scenarios[sc]], sigma=False, fixed_point_bits=34)
            qd, _ = eng.last_tally(0)
            dense += qd.cpu().numpy().ravel()
        acc = np.zeros(g.nvox, np.int64)
        for r in range(sc * n_per_scen, (sc + 1) * n_per_scen):
            cc, qq = rows[r]
            assert np.all(np.diff(cc) > 0)
            np.add.at(acc, cc, qq)
        assert dense.any() and np.array_equal(acc, dense)


@pytest.mark.gpu
def test_atomic_rate_microbenchmark():
    """The roofline's atomic-rate probe runs on the device and reports a
    plausible rate for the head grid's shape (int64 adds per second)."""
    from paper_2307_01416_amd import vpmc as V
    c = V.vpmc_create(0)
    try:
        r = V.vpmc_atomic_rate(c, (256, 256, 160), 1 << 22)
    finally:
        V.vpmc_destroy(c)
    print(f"  int64 atomic adds: {r:.3e} per second")
    assert 1e8 < r < 1e13
