"""The robust influence-matrix pass at its full size, in the launch shape the
throughput measurement times: the synthetic head CT (256 x 256 x 160 voxels
of 1 x 1 x 2 mm), three fields of 950 spots, 13 robust scenarios (37 050
rows), 19 520 VPs per spot nominal (uneven across spots: 19 289 on average,
7.15e8 per pass), 2 histories per lane, 256 workgroups of 1024 threads.

Straight mode (the deterministic parity bar, 1e-5 relative per voxel):
sampled rows of the first field equal the oracle's single-spot tallies,
outside the voxels an FP32/FP64 rounding of the source position could move.
The sampled scenarios shift the isocentre along the beam or by whole voxels
across it, at both range scalings, so the lateral voxel boundaries the
rounding test uses are known.

Full physics (properties that hold at any size): columns ascend in every
row, and the rows of each sampled scenario sum to the dense tallies of its
three fields bit for bit."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from test_gpu_parity import ambiguous_mask, assert_straight_parity, say

pytestmark = pytest.mark.gpu

VPS_PER_SPOT = 19_520
SHAPE = dict(hist_per_lane=2, grid_blocks=256, block_threads=1024)


@pytest.fixture(scope="module")
def eng():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    e = V.Engine(0)
    yield e
    e.close()


def full_run(eng, case):
    """The whole pass; returns (host row_ptr, device col, device q, k)."""
    import torch
    from paper_2307_01416_amd import vpmc as V
    rp, col, val, _, k = eng.run_csr(case, device_out=True, **SHAPE)
    del val
    q = torch.empty(col.numel(), dtype=torch.int64, device=col.device)
    V.vpmc_copy_csr(eng.ctx, None, None, q)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col, q, k


def test_full_size_straight_rows_equal_oracle(eng, orc):
    import torch
    case = I.config4(8.0, VPS_PER_SPOT, physics=0)
    n_rows = len(case.scenarios) * sum(len(f.spots) for f in case.fields)
    assert n_rows == 37_050 and case.geometry.shape == (256, 256, 160)
    say(f"full-size straight: rows {n_rows}, VPs {sum(int(f.spots['n_histories'].sum()) for f in case.fields) * 13}")
    rp, col, q, k = full_run(eng, case)
    say(f"  nnz {int(rp[-1])}, k {k}")
    n_per_scen = sum(len(f.spots) for f in case.fields)
    nz, ny, nx = case.geometry.shape[2], case.geometry.shape[1], case.geometry.shape[0]
    # field 0's beam runs along -x: shifts along x or by whole 1 mm voxels along y
    assert tuple(case.fields[0].beam.ez) == (-1.0, 0.0, 0.0)
    samples = [(0, 0), (0, 949), (2, 317), (5, 633), (8, 158), (4, 800)]
    for sc, sp in samples:
        sh = case.scenarios[sc].shift_mm
        assert sh[2] == 0.0 and float(sh[1]).is_integer()
        r = sc * n_per_scen + sp
        a, b = int(rp[r]), int(rp[r + 1])
        cc = col[a:b].cpu().numpy()
        qq = q[a:b].cpu().numpy()
        assert b > a and np.all(np.diff(cc) > 0)
        qg = np.zeros(nz * ny * nx, np.int64)
        qg[cc] = qq
        qo, _, ko = orc.run_tally(case, field_index=0, scenario_index=sc, k=k, spots=(sp, sp + 1))
        say(f"  row scenario {sc} spot {sp}: {b - a} entries")
        assert_straight_parity(qg.reshape(nz, ny, nx), k, qo, ko,
                               ambiguous_mask(orc, case, spots=[sp], shift_mm=sh))
    del col, q
    torch.cuda.empty_cache()


def test_full_size_physics_rows_sum_to_dense(eng):
    import torch
    case = I.config4(8.0, VPS_PER_SPOT)
    say("full-size full physics: 37 050 rows")
    rp, col, q, k = full_run(eng, case)
    say(f"  nnz {int(rp[-1])}, k {k}")
    n_per_scen = sum(len(f.spots) for f in case.fields)
    nvox = case.geometry.nvox
    for sc in (0, 10):
        a, b = int(rp[sc * n_per_scen]), int(rp[(sc + 1) * n_per_scen])
        cc = col[a:b].cpu().numpy()
        qq = q[a:b].cpu().numpy()
        starts = rp[sc * n_per_scen:(sc + 1) * n_per_scen + 1] - a
        # ascending columns within every row (a decrease only where a row starts)
        down = np.nonzero(np.diff(cc) <= 0)[0] + 1
        assert np.isin(down, starts).all()
        acc = np.zeros(nvox, np.int64)
        np.add.at(acc, cc, qq)
        del cc, qq
        dense = np.zeros(nvox, np.int64)
        for fi in range(len(case.fields)):
            eng.run_dose(case, fi, scenarios=[case.scenarios[sc]], sigma=False, fixed_point_bits=k)
            qd, kd = eng.last_tally(0)
            assert kd == k
            dense += qd.cpu().numpy().ravel()
        say(f"  scenario {sc}: {b - a} entries, dense sum {int(dense.sum())}")
        assert dense.any() and np.array_equal(acc, dense)
    del col, q
    torch.cuda.empty_cache()
