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
row, the rows of each sampled scenario sum to the dense tallies of its three
fields bit for bit, the dynamic-spacing merge of the whole IM keeps every
row's exact total, the optimiser's reported objective matches its weights,
the LET tally leaves the dose tally unchanged, and the divergent and
energy-layer aperture IMs sum to their dense tallies.  The learned
surrogate's plan dose is compared with a plain run statistically."""
import numpy as np
import pytest

from paper_2307_01416_amd import inputs as I
from straight_bound import allowance, assert_straight_parity
from test_gpu_parity import say

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
    """The whole pass; returns (host row_ptr, device col, device FP32 Gy
    values, device int64 tallies, k)."""
    import torch
    from paper_2307_01416_amd import vpmc as V
    rp, col, val, _, k = eng.run_csr(case, device_out=True, **SHAPE)
    q = torch.empty(col.numel(), dtype=torch.int64, device=col.device)
    V.vpmc_copy_csr(eng.ctx, None, None, q)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col, val, q, k


def test_full_size_straight_rows_equal_oracle(eng, orc):
    import torch
    case = I.config4(8.0, VPS_PER_SPOT, physics=0)
    n_rows = len(case.scenarios) * sum(len(f.spots) for f in case.fields)
    assert n_rows == 37_050 and case.geometry.shape == (256, 256, 160)
    say(f"full-size straight: rows {n_rows}, VPs {sum(int(f.spots['n_histories'].sum()) for f in case.fields) * 13}")
    rp, col, val, q, k = full_run(eng, case)
    del val
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
        allow, n_amb = allowance(orc, case, 0, sc, spots=[sp])
        say(f"    {n_amb} histories near a boundary")
        assert_straight_parity(qg.reshape(nz, ny, nx), k, qo, ko, allow, say=say)
    del col, q
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def physics_pass(eng):
    import torch
    case = I.config4(8.0, VPS_PER_SPOT)
    say("full-size full physics: 37 050 rows")
    rp, col, val, q, k = full_run(eng, case)
    say(f"  nnz {int(rp[-1])}, k {k}")
    yield case, rp, col, val, q, k
    del col, val, q
    torch.cuda.empty_cache()


def row_totals(rp, q, r0, r1):
    """Exact int64 totals of rows r0 .. r1-1 (host row_ptr, device values)."""
    a, b = int(rp[r0]), int(rp[r1])
    qq = q[a:b].cpu().numpy()
    lens = np.diff(rp[r0:r1 + 1])
    out = np.zeros(r1 - r0, np.int64)
    nz = lens > 0
    if qq.size:
        out[nz] = np.add.reduceat(qq, (rp[r0:r1] - a)[nz])
    return out


def test_full_size_physics_rows_sum_to_dense(eng, physics_pass):
    case, rp, col, _, q, k = physics_pass
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


def test_full_size_dynamic_spacing_conserves_rows(eng, physics_pass):
    """The cell merge of the whole IM (target voxels kept, organ at risk in
    runs of 2, other voxels in runs of 4 along x): every row keeps its exact
    int64 total, cells ascend within each row and stay below n_cells."""
    import torch
    from paper_2307_01416_amd import vpmc as V
    case, rp, col, _, q, k = physics_pass
    roi = I.head_structures(case, 8.0)
    cmap, n_cells = I.dynamic_spacing_map(case.geometry.shape, roi, target=1, oar=2, other=4)
    dev = col.device
    rpd = torch.from_numpy(rp).to(dev)
    rpc, cell, qc, val = V.vpmc_csr_cells(eng.ctx, rpd, col, q, k, torch.from_numpy(cmap).to(dev), n_cells,
                                          V.DEVICE_PTRS)
    torch.cuda.synchronize()
    rpc = rpc.cpu().numpy()
    say(f"  cells: {n_cells} for {case.geometry.nvox} voxels, entries {int(rp[-1])} -> {int(rpc[-1])}")
    assert int(rpc[-1]) < int(rp[-1])
    assert int(torch.sum(q).item()) == int(torch.sum(qc).item())
    n_per_scen = sum(len(f.spots) for f in case.fields)
    for sc in (0, 10):
        r0, r1 = sc * n_per_scen, (sc + 1) * n_per_scen
        assert np.array_equal(row_totals(rp, q, r0, r1), row_totals(rpc, qc, r0, r1))
        a, b = int(rpc[r0]), int(rpc[r1])
        cc = cell[a:b].cpu().numpy()
        assert cc.size == 0 or (cc.min() >= 0 and cc.max() < n_cells)
        down = np.nonzero(np.diff(cc) <= 0)[0] + 1
        assert np.isin(down, rpc[r0:r1 + 1] - a).all()
    del rpc, cell, qc, val
    torch.cuda.empty_cache()


def test_full_size_optimiser_objective_matches_its_weights(eng, physics_pass):
    """Spot-weight optimisation on the whole 13-scenario IM as the throughput
    measurement runs it (start scaled to the prescription, 20 power and 80
    FISTA iterations): the objective reported at the final weights equals the
    objective recomputed from those weights and the same matrices in FP64
    (the optimiser's dose sums are int64 fixed point at 2^-60 of their
    bound: 1e-8 relative), its dose output equals the recomputed dose to
    1e-6 of the maximum (FP32 output), and the objective falls."""
    import torch
    from paper_2307_01416_amd import vpmc as V
    case, rp, col, val, _, _ = physics_pass
    n_scen = len(case.scenarios)
    n_spots = sum(len(f.spots) for f in case.fields)
    nvox = case.geometry.nvox
    dev = col.device
    rpd = torch.from_numpy(rp).to(dev)
    roi = torch.from_numpy(I.head_structures(case, 8.0)).to(dev)
    par = dict(d_presc=2.0, w_target=1.0, d_max=1.0, w_oar=1.0)
    dose = torch.empty((n_scen, nvox), dtype=torch.float32, device=dev)
    x = torch.ones(n_spots, dtype=torch.float64, device=dev)
    V.vpmc_optimize(eng.ctx, rpd, col, val, n_scen, n_spots, nvox, roi, x, iters=0, n_power=1,
                    flags=V.DEVICE_PTRS, dose=dose, **par)
    tm, om = (roi & 1) > 0, (roi & 2) > 0
    x = torch.full((n_spots,), par["d_presc"] / float(dose[:, tm].mean()), dtype=torch.float64, device=dev)
    hist = torch.zeros(81, dtype=torch.float64, device=dev)
    L = V.vpmc_optimize(eng.ctx, rpd, col, val, n_scen, n_spots, nvox, roi, x, iters=80, n_power=20,
                        flags=V.DEVICE_PTRS | V.OPT_REUSE, obj_hist=hist, dose=dose, **par)
    torch.cuda.synchronize()
    hist = hist.cpu().numpy()
    assert L > 0 and bool((x >= 0).all())
    F = 0.0
    dmax_err = 0.0
    for s in range(n_scen):
        r0, r1 = s * n_spots, (s + 1) * n_spots
        a, b = int(rp[r0]), int(rp[r1])
        lens = torch.from_numpy(np.diff(rp[r0:r1 + 1])).to(dev)
        w = torch.repeat_interleave(x, lens)
        D = torch.zeros(nvox, dtype=torch.float64, device=dev)
        D.index_add_(0, col[a:b].long(), val[a:b].double() * w)
        del w
        dt = D[tm] - par["d_presc"]
        do = torch.clamp(D[om] - par["d_max"], min=0.0)
        F += par["w_target"] * float((dt * dt).sum()) + par["w_oar"] * float((do * do).sum())
        dmax_err = max(dmax_err, float((dose[s].double() - D).abs().max() / D.max()))
    F /= n_scen
    say(f"  optimiser on the full IM: F {hist[0]:.4f} -> {hist[-1]:.4f}, recomputed {F:.4f}, "
        f"dose max err {dmax_err:.2e} of max, L {L:.4e}")
    assert hist[-1] == pytest.approx(F, rel=1e-8)
    assert dmax_err <= 1e-6
    assert hist[-1] < 0.2 * hist[0]


def test_full_size_let_leaves_the_dose_tally_unchanged(eng, orc):
    """The nominal plan of the full head case (three fields at the full VPs
    per spot, full physics): each field's dose tally with the LET numerator
    tallied beside it equals the tally without it bit for bit, and the plan's
    LET_d per unit density (a dose-weighted mean of the steps' mass stopping
    powers) lies within the range of those: about 0.4 keV/um per g/cm3 at
    230 MeV up to about 30 for the last step below the 1 MeV cut-off (the
    slope of the range table's first segment), checked as (0.3, 40) wherever
    there is dose."""
    case = I.config4(8.0, VPS_PER_SPOT)
    nom = I.Case("nominal", case.geometry, case.fields, [I.Scenario()], seed=case.seed, physics=case.physics)
    eng.load_case(nom)
    q_sum = ql_sum = None
    for fi in range(len(nom.fields)):
        eng.run_dose(nom, fi, n_batches=0, sigma=False, let=False, fixed_point_bits=36)
        q0, _ = eng.last_tally(0)
        q0 = q0.cpu().numpy()
        eng.run_dose(nom, fi, n_batches=0, sigma=False, let=True, fixed_point_bits=36)
        q1, k = eng.last_tally(0)
        ql, sh = eng.last_let(0)
        q1, ql = q1.cpu().numpy(), ql.cpu().numpy()
        say(f"  field {fi}: dose voxels {int((q1 > 0).sum())}, LET shift {sh}")
        assert q1.any() and np.array_equal(q0, q1)
        q_sum = q1.astype(np.float64) if q_sum is None else q_sum + q1
        part = ql.astype(np.float64) * 2.0 ** sh
        ql_sum = part if ql_sum is None else ql_sum + part
    _, rho = orc.hu_lookup(case.geometry.hu)
    rho = np.asarray(rho, np.float64).reshape(q_sum.shape)
    m = q_sum > 1e-3 * q_sum.max()
    let_d = ql_sum[m] / q_sum[m]
    mass_let = let_d / rho[m]
    say(f"  plan LET_d over {int(m.sum())} voxels: {let_d.min():.3f} - {let_d.max():.3f} keV/um, "
        f"per unit density {mass_let.min():.3f} - {mass_let.max():.3f}")
    assert mass_let.min() > 0.3 and mass_let.max() < 40.0


@pytest.mark.parametrize("variant", ["divergent", "layer_apertures"])
def test_full_size_variant_rows_sum_to_dense(eng, variant):
    """The two aperture variants as the throughput measurement builds their
    IMs: beam from a virtual source 2 m upstream with the blocks' walls
    focused on it, and one 32-vertex aperture per energy layer (30 fields).
    The rows of the nominal scenario sum to the dense tallies of all fields
    bit for bit, and columns ascend in every row."""
    import torch
    layers = variant == "layer_apertures"
    case = I.config4(8.0, VPS_PER_SPOT, layer_apertures=layers, n_vertices=32 if layers else 128)
    if not layers:
        for f in case.fields:
            f.vsad_mm = 2000.0
            f.block.focus_mm = 2000.0
    rp, col, val, q, k = full_run(eng, case)
    del val
    n_per_scen = sum(len(f.spots) for f in case.fields)
    assert n_per_scen * len(case.scenarios) == 37_050
    a, b = int(rp[0]), int(rp[n_per_scen])
    cc = col[a:b].cpu().numpy()
    qq = q[a:b].cpu().numpy()
    del col, q
    torch.cuda.empty_cache()
    down = np.nonzero(np.diff(cc) <= 0)[0] + 1
    assert np.isin(down, rp[:n_per_scen + 1] - a).all()
    nvox = case.geometry.nvox
    acc = np.zeros(nvox, np.int64)
    np.add.at(acc, cc, qq)
    del cc, qq
    dense = np.zeros(nvox, np.int64)
    for fi in range(len(case.fields)):
        eng.run_dose(case, fi, scenarios=[case.scenarios[0]], sigma=False, fixed_point_bits=k)
        qd, kd = eng.last_tally(0)
        assert kd == k
        dense += qd.cpu().numpy().ravel()
    say(f"  {variant}: fields {len(case.fields)}, nnz {int(rp[-1])}, nominal rows {b - a} entries")
    assert dense.any() and np.array_equal(acc, dense)


def plan_dose(eng, case, seed, surrogate=False, mult=4):
    """Nominal uniform-weight plan dose of all fields at mult x the VPs per
    spot and its batch standard error (16 batches), FP64 numpy."""
    fields = [I.Field(beam=f.beam, spots=f.spots.copy(), polygon=f.polygon, block=f.block, rs=f.rs,
                      vsad_mm=f.vsad_mm) for f in case.fields]
    for f in fields:
        f.spots["n_histories"] = (f.spots["n_histories"].astype(np.uint64) * mult).astype(np.uint32)
    nom = I.Case("nominal", case.geometry, fields, [I.Scenario()], seed=case.seed, physics=case.physics,
                 n_batches=16)
    eng.load_case(nom)
    total = var = None
    for fi in range(len(nom.fields)):
        d, s, _ = eng.run_dose(nom, fi, n_batches=16, sigma=True, seed=seed, surrogate=surrogate)
        d, s = d[0].double().cpu().numpy(), s[0].double().cpu().numpy()
        total = d if total is None else total + d
        var = s * s if var is None else var + s * s
    return total, np.sqrt(var)


def test_full_size_surrogate_plan_dose(eng):
    """The learned aperture surrogate on the full head case, as the
    throughput measurement compares it: trained on the GPU on plain brass
    traversals near the three apertures' edges (3e6 samples, 6 epochs), the
    nominal plan dose of the three fields at 4x the VPs per spot (U about
    0.25 %) with the surrogate against an independent plain run: >= 99 % of
    the voxels >= 10 % of the maximum within 3 combined standard errors,
    gamma 1 %/1 mm >= 99 % (global, 10 % threshold), mean over the
    high-dose region within 0.5 %."""
    from gamma import gamma_pass_rate
    from paper_2307_01416_amd import vpmc as V
    case = I.config4(8.0, VPS_PER_SPOT)
    losses = eng.train_surrogate(case, n=3_000_000, epochs=6, seed=3, fields=range(len(case.fields)))
    assert losses[-1] < losses[0]
    V.vpmc_surrogate_config(eng.ctx)
    dp, sp = plan_dose(eng, case, seed=case.seed + 101)
    ds, ss = plan_dose(eng, case, seed=case.seed + 202, surrogate=True)
    m = dp >= 0.1 * dp.max()
    frac = float(np.mean(np.abs(ds - dp)[m] <= 3.0 * np.sqrt(sp ** 2 + ss ** 2)[m]))
    avg = 0.5 * (dp + ds)
    hi = avg >= 0.5 * avg.max()
    ratio = float(ds[hi].mean() / dp[hi].mean())
    idx = np.nonzero(m)
    box = tuple(slice(max(0, int(i.min()) - 2), int(i.max()) + 3) for i in idx)
    rate = gamma_pass_rate(dp[box], ds[box], case.geometry.spacing, 0.01, 1.0)
    say(f"  surrogate vs plain at full size: losses {losses[0]:.4f} -> {losses[-1]:.4f}, 3-sigma {frac:.4f}, "
        f"gamma 1%/1mm {rate:.4f}, high-dose mean ratio {ratio:.5f}")
    assert frac >= 0.99 and rate >= 0.99 and abs(ratio - 1.0) <= 0.005
