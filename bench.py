"""Benchmark of the VP transport on one MI355X: the 13-scenario influence
matrix of the synthetic head case.

Workload (one step): synthetic head CT 256x256x160 at 1x1x2 mm, 8 cc
spherical target, 3 coplanar fields each with a 30 mm brass aperture
(target projection + 5 mm) and a 45 mm WET PMMA range shifter, ~950 spots per
field on a 2.5 mm grid, 13 robust scenarios (nominal + +-3 mm shifts along
x/y/z at +-3.5 % range), uneven history counts per spot.  One batched
work-queue pass builds all 13 x 3 x spots sparse rows in HBM, converted to
device-resident CSR (int32 voxel, FP32 Gy per unit spot weight).  History counts are scaled before timing until the nominal
uniform-weight plan dose has a mean relative standard error <= 0.5 % over
voxels >= 50 % of its maximum.  Inputs are synthetic and resident on the GPU
before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per condensed-history step counted from the method
# (about 300): Philox4x32-10 ~100 integer ops, uniform conversions 8,
# normal quantile 25, Box-Muller with log/sqrt/sin/cos at quarter rate 22,
# energy-segment search and four table interpolations 35, CSDA loss 12,
# hinge rotation 35, voxel traversal (three face distances, index update) 25,
# nuclear test 8, fixed-point tally 8, position and energy updates 12,
# range-out and step-length logic 10
ALG_OPS_PER_STEP = 300.0
# gfx950: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one VALU lane-operation per
# lane and clock (non-packed; packed FP32 is switched off at build time)
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# the published FP32 vector peak (packed FMA: 2 flops x 2 per lane and clock)
FP32_PEAK_FLOPS = 157.3e12
# wave64 VALU instructions issued per second over the chip: 1024 SIMDs, 4
# clocks each
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4.0
HBM_PEAK = 8.0e12   # MI355X HBM3E, bytes/s
TARGET_U = 0.005


PROFILE = os.path.join(ROOT, "profiles", "queue_kernel_head_im.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2307_01416_amd", "csrc", "vpmc_kernels.hip")
BUILD_SCRIPT = os.path.join(ROOT, "paper_2307_01416_amd", "build.py")


OPT_PROFILE = os.path.join(ROOT, "profiles", "optimizer_head_im.md")
OPT_SRC = os.path.join(ROOT, "paper_2307_01416_amd", "csrc", "vpmc_opt.hip")


def measured_traffic(profile=PROFILE, src_path=KERNEL_SRC, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of queue_kernel (or per optimiser iteration) from a
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated
    on a plain copy), or None when the kernel source has changed since the
    counters were taken."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        src = hashlib.sha256(open(src_path, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(key + r":\s*([0-9.eE+]+)", text)
    h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != src:
        return None
    # counters that depend on the code generation also name the build script
    # (its compiler flags) they were taken with
    b = re.search(r"build_sha256:\s*([0-9a-f]{64})", text)
    if b and b.group(1) != hashlib.sha256(open(BUILD_SCRIPT, "rb").read()).hexdigest():
        return None
    return float(m.group(1))


def progress(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--target-cc", type=float, default=8.0)
    ap.add_argument("--histories-per-spot", type=float, default=1e4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", action="store_true", help="capture the pass in one hipGraph")
    ap.add_argument("--no-scale", action="store_true",
                    help="keep --histories-per-spot as given (skip the scaling to 0.5 %% uncertainty)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate comparison")
    ap.add_argument("--no-per-spot", action="store_true", help="skip the per-spot plain-launch baseline")
    ap.add_argument("--sur-samples", type=int, default=200_000_000,
                    help="entry states near the edges (about half cross brass and train the network)")
    ap.add_argument("--sur-epochs", type=int, default=2)
    ap.add_argument("--no-optimize", action="store_true", help="skip the spot-weight optimiser measurement")
    ap.add_argument("--let", action="store_true",
                    help="also time the nominal plan dose with and without the dose-averaged LET tally")
    ap.add_argument("--dynamic-spacing", action="store_true",
                    help="also merge the head IM into coarser cells away from the target (dynamic voxel spacing)")
    ap.add_argument("--layer-apertures", action="store_true",
                    help="energy-layer-specific apertures: one field per energy layer (30 fields)")
    ap.add_argument("--divergent", type=float, default=0.0, metavar="MM",
                    help="virtual source and block focus this far upstream of the isocentre (0: off)")
    ap.add_argument("--opt-iters", type=int, default=80)
    ap.add_argument("--shape", default="", help="HPL,BLOCKS,THREADS: fixed work-queue launch shape (no autotune)")
    ap.add_argument("--oracle-suite", action="store_true",
                    help="time the oracle beside the GPU on config 1 and two config-2 cases (not the bench line)")
    ap.add_argument("--resolution-study", action="store_true",
                    help="the head IM on 1x1x2, 1x1x1 and 2x2x2 mm grids and the coarse doses' gamma against "
                         "1 mm (not the bench line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="before the workload, run three plain 256 MiB device copies (HBM counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """Three device-to-device copies of 256 MiB: a kernel of known traffic
    (256 MiB read + 256 MiB written) for scaling the HBM byte counters."""
    import torch
    n = 1 << 26
    a = torch.arange(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    progress(f"copy calibration: 3 x {4 * n >> 20} MiB copies done")
    del a, b


def plan_dose(eng, case, I, seed=None, surrogate=False, mult=1):
    """Nominal uniform-weight plan dose of all fields and its batch standard
    error (16 batches), as FP64 torch tensors on the GPU; mult scales every
    spot's history count."""
    import numpy as np
    import torch
    fields = case.fields
    if mult != 1:
        fields = [I.Field(beam=f.beam, spots=f.spots.copy(), polygon=f.polygon, block=f.block, rs=f.rs,
                          vsad_mm=f.vsad_mm) for f in case.fields]
        for f in fields:
            f.spots["n_histories"] = (f.spots["n_histories"].astype(np.uint64) * mult).astype(np.uint32)
    nom = I.Case("nominal", case.geometry, fields, [I.Scenario()], seed=case.seed, physics=case.physics,
                 n_batches=16)
    eng.load_case(nom)
    total = None
    var = None
    for fi in range(len(nom.fields)):
        d, s, _ = eng.run_dose(nom, fi, n_batches=16, sigma=True, seed=seed, surrogate=surrogate)
        d = d[0].double()
        s = s[0].double()
        total = d if total is None else total + d
        var = s * s if var is None else var + s * s
    return total, torch.sqrt(var)


def plan_uncertainty(eng, case, I, V, np):
    """U of the nominal uniform-weight plan dose (all fields, 16 batches):
    mean sigma/D over voxels >= 50 % of the maximum."""
    total, sig = plan_dose(eng, case, I)
    m = total >= 0.5 * total.max()
    return float((sig[m] / total[m]).mean())


def surrogate_comparison(eng, case, I, V, np, a, shape, plain_s, plain_steps):
    """The learned aperture surrogate on the same influence matrices: train
    it on the GPU (plain brass traversals near the three apertures' edges,
    a.sur_samples of them), then time the 13-scenario IM with it exactly as
    the plain one was timed (a.warmup untimed, a.steps timed), and compare the
    nominal plan dose with and without it (independent seeds, 4x the IM's
    histories): fraction of voxels >= 10 % of the maximum within 3 combined
    standard errors, gamma 1 %/1 mm (global, 10 % threshold), high-dose mean
    ratio; a second plain run gives the gamma noise floor."""
    import torch
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gamma import gamma_pass_rate
    t0 = time.perf_counter()
    losses = eng.train_surrogate(case, n=a.sur_samples, epochs=a.sur_epochs, seed=3,
                                 fields=range(len(case.fields)))
    train_s = time.perf_counter() - t0
    progress(f"surrogate trained on {a.sur_samples:.3g} traversals in {train_s:.1f} s, "
             f"losses {[round(float(x), 4) for x in losses]}")
    V.vpmc_surrogate_config(eng.ctx)
    eng.load_case(case)
    for _ in range(a.warmup):
        _, col, val, _, _ = eng.run_csr(case, device_out=True, surrogate=True, **shape)
        del col, val
    torch.cuda.synchronize()
    sts = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, col, val, _, _ = eng.run_csr(case, device_out=True, surrogate=True, **shape)
        sts.append(V.vpmc_last_stats(eng.ctx))
        del col, val
    torch.cuda.synchronize()
    sur_s = (time.perf_counter() - t0) / a.steps
    deferred = sum(st["deferred"] for st in sts) / a.steps
    hist = sum(st["histories"] for st in sts) / a.steps
    steps = sum(st["steps"] for st in sts) / a.steps
    progress(f"IM with surrogate: {sur_s:.3f} s (plain {plain_s:.3f} s), deferred {deferred:.0f} of {hist:.0f}")
    # accuracy at 4x the influence matrix's histories (U ~ 0.25 %), against an
    # independent plain run; a second plain run gives the noise floor
    dp, sp = plan_dose(eng, case, I, seed=case.seed + 101, mult=4)
    ds, ss = plan_dose(eng, case, I, seed=case.seed + 202, surrogate=True, mult=4)
    d2, _ = plan_dose(eng, case, I, seed=case.seed + 303, mult=4)
    dp, sp, ds, ss, d2 = (t.cpu().numpy() for t in (dp, sp, ds, ss, d2))
    m = dp >= 0.1 * dp.max()
    frac = float(np.mean(np.abs(ds - dp)[m] <= 3.0 * np.sqrt(sp ** 2 + ss ** 2)[m]))
    hi = dp >= 0.5 * dp.max()
    ratio = float(ds[hi].mean() / dp[hi].mean())
    # gamma on the bounding box of the 10 % region (+2 voxels)
    idx = np.nonzero(m)
    box = tuple(slice(max(0, int(i.min()) - 2), int(i.max()) + 3) for i in idx)
    rate = gamma_pass_rate(dp[box], ds[box], case.geometry.spacing, 0.01, 1.0)
    floor = gamma_pass_rate(dp[box], d2[box], case.geometry.spacing, 0.01, 1.0)
    progress(f"surrogate vs plain: 3-sigma {frac:.4f}, gamma 1%/1mm {rate:.4f} (plain vs plain {floor:.4f}), "
             f"mean ratio {ratio:.5f}")
    return {"s_per_13_scenario_im": sur_s, "speedup_vs_plain": plain_s / sur_s,
            "deferred_fraction": deferred / max(1.0, hist), "training_s": train_s,
            "training_traversals": a.sur_samples, "epochs": a.sur_epochs,
            "plan_dose_3sigma_fraction": frac, "plan_dose_gamma_1pct_1mm": rate,
            "plan_dose_gamma_plain_vs_plain": floor, "plan_dose_mean_ratio": ratio, "plan_dose_histories_x": 4,
            "steps_ratio": steps / max(1.0, plain_steps), "timed_steps": a.steps, "warmup": a.warmup}


def per_spot_baseline(eng, case, I, V, np, stride=50):
    """The influence matrices as one plain launch per row (one vpmc_run_spots
    call in CSR mode per scenario x field x spot, the way a per-spot engine
    builds them): every stride-th row is run and timed, and the time of the
    whole matrix is extrapolated from their mean."""
    import torch
    eng.load_case(case)
    rows = [(s, f, j) for s in range(len(case.scenarios)) for f in range(len(case.fields))
            for j in range(len(case.fields[f].spots))]
    sample = rows[::stride]
    rp = np.zeros(2, np.int64)
    led = np.zeros((1, V.NLEDGER))

    def one(s, f, j):
        spot = case.fields[f].spots[j:j + 1]
        opts = V.make_opts(seed=case.seed, physics=case.physics, output=V.OUT_CSR, stream=eng.stream_ptr())
        V.vpmc_run_spots(eng.ctx, f, V.spot_array(spot), 1, V.scenario_array([case.scenarios[s]]), 1, opts,
                         None, None, led, rp)

    one(*sample[0])   # warm-up (buffers sized)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in sample:
        one(*r)
    torch.cuda.synchronize()
    per_row = (time.perf_counter() - t0) / len(sample)
    progress(f"per-spot plain launches: {1e3 * per_row:.2f} ms per row over {len(sample)} sampled rows, "
             f"{per_row * len(rows):.1f} s per IM extrapolated")
    return {"s_per_13_scenario_im_extrapolated": per_row * len(rows), "ms_per_row": 1e3 * per_row,
            "rows_timed": len(sample), "rows": len(rows),
            "what": "one vpmc_run_spots call (CSR, one spot, one scenario) per row, rows sampled every "
                    f"{stride}th, same histories and seed, time extrapolated to all rows"}


def optimizer_measure(eng, case, I, V, np, torch, a, shape):
    """Robust spot-weight optimisation on the head case's 13-scenario
    influence matrices (device CSR): index build, then the time per FISTA
    iteration from two calls on the reused index (difference of
    a.opt_iters and a.opt_iters // 4 iterations), HBM-bound roofline of an
    iteration (the entries in structure voxels read twice, the structure
    voxels' residual written and read once and their mask read once per
    scenario)."""
    rp, col, val, _, _ = eng.run_csr(case, device_out=True, **shape)
    dev = col.device
    n_scen = len(case.scenarios)
    n_spots = sum(len(fl.spots) for fl in case.fields)
    nvox = case.geometry.nvox
    nnz = int(col.numel())
    roi = torch.from_numpy(I.head_structures(case, a.target_cc)).to(dev)
    par = dict(d_presc=2.0, w_target=1.0, d_max=1.0, w_oar=1.0)
    x = torch.ones(n_spots, dtype=torch.float64, device=dev)
    dose = torch.empty((n_scen, nvox), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V.vpmc_optimize(eng.ctx, rp, col, val, n_scen, n_spots, nvox, roi, x, iters=0, n_power=1,
                    flags=V.DEVICE_PTRS, stream=eng.stream_ptr(), dose=dose, **par)
    t_first = time.perf_counter() - t0
    tmask = (roi & 1) > 0
    scale = par["d_presc"] / float(dose[:, tmask].mean())
    runs = {}
    for iters in (a.opt_iters // 4, a.opt_iters):
        x = torch.full((n_spots,), scale, dtype=torch.float64, device=dev)
        hist = torch.zeros(iters + 1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = V.vpmc_optimize(eng.ctx, rp, col, val, n_scen, n_spots, nvox, roi, x, iters=iters, n_power=20,
                            flags=V.DEVICE_PTRS | V.OPT_REUSE, stream=eng.stream_ptr(), obj_hist=hist,
                            dose=dose, **par)
        runs[iters] = (time.perf_counter() - t0, hist.cpu().numpy(), L)
        progress(f"optimiser: {iters} iterations in {runs[iters][0]:.3f} s")
    i1, i2 = a.opt_iters // 4, a.opt_iters
    t_it = (runs[i2][0] - runs[i1][0]) / (i2 - i1)
    hist = runs[i2][1]
    dt = dose[:, tmask]
    do = dose[:, (roi & 2) > 0]
    # entries in structure voxels (the iterations' working set) and the
    # structure voxels: each entry is read twice per iteration (dose and
    # gradient sweeps), each structure voxel's residual written and read once
    # per scenario, its mask byte read once per scenario
    n_roi_entries = int(sum(int((roi[col[i:i + (1 << 28)].long()] != 0).sum())
                            for i in range(0, nnz, 1 << 28)))
    n_roi_vox = int((roi != 0).sum())
    alg = 16.0 * n_roi_entries + n_scen * n_roi_vox * (4.0 + 4.0 + 1.0)
    del rp, col, val
    return {"what": "robust spot-weight optimisation (projected FISTA, 13 scenarios, target + organ-at-risk "
                    "quadratic penalties) on the device-resident influence matrices",
            "n_spots": n_spots, "nnz": nnz, "structure_entries": n_roi_entries, "structure_voxels": n_roi_vox,
            "index_build_and_first_call_s": t_first,
            "iters": i2, "s_total": runs[i2][0], "ms_per_iteration": 1e3 * t_it, "step_L": runs[i2][2],
            "objective_first": float(hist[0]), "objective_final": float(hist[-1]),
            "target_mean_dose_gy_per_scenario_min_max": [float(dt.mean(1).min()), float(dt.mean(1).max())],
            "oar_max_dose_gy_worst_scenario": float(do.max()),
            "roofline": {"bound": "hbm", "achieved": alg / t_it / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": alg / t_it / HBM_PEAK,
                         "traffic": measured_traffic(OPT_PROFILE, OPT_SRC, "traffic_bytes_per_iteration"),
                         "kernel": "opt_forward_kernel + opt_grad_kernel (one iteration)",
                         "alg_bytes_per_iteration": alg}}


def dynamic_spacing_measure(eng, case, I, V, np, torch, a, shape):
    """Dynamic voxel spacing (coarser IM cells away from the target) of the
    head IM: rows merged into cells of 1 (target), 2 (organ at risk) and 4 or
    8 (elsewhere) voxels along x, on the device; cells, entries, time of the
    merge (both passes, map checks included)."""
    rp, col, val, _, _ = eng.run_csr(case, device_out=True, **shape)
    k = V.vpmc_last_tally_k(eng.ctx)
    nnz = int(col.numel())
    del val
    q = torch.empty(nnz, dtype=torch.int64, device=col.device)
    V.vpmc_copy_csr(eng.ctx, None, None, q)
    roi = I.head_structures(case, a.target_cc)
    out = {"nnz_voxels": nnz}
    for other in (4, 8):
        cmap, n_cells = I.dynamic_spacing_map(case.geometry.shape, roi, target=1, oar=2, other=other)
        cm = torch.from_numpy(cmap).to(col.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rpc, cell, qc, valc = V.vpmc_csr_cells(eng.ctx, rp, col, q, k, cm, n_cells, V.DEVICE_PTRS)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_out = int(cell.numel())
        out[f"target1_oar2_other{other}"] = {"cells": n_cells, "entries": n_out, "entries_ratio": n_out / nnz,
                                             "gb_int32_fp32": 8e-9 * n_out, "s_merge": dt}
        progress(f"dynamic spacing (other {other}): {n_cells} cells, {n_out} entries ({n_out / nnz:.3f} of "
                 f"{nnz}) in {dt:.3f} s")
        del rpc, cell, qc, valc, cm
    del rp, col, q
    return out


def let_measure(eng, case, I, V, np, torch, a):
    """Dose-averaged LET tally on the head case: the nominal plan dose of all
    fields (dense, no batches) with and without the LET numerator (one more
    int64 tally per step), twice each, interleaved; the plan's LET_d in the
    target and the organ at risk (sum over fields of the numerators over the
    sum of the dose tallies, the same k for every field)."""
    nom = I.Case("nominal", case.geometry, case.fields, [I.Scenario()], seed=case.seed, physics=case.physics)
    eng.load_case(nom)
    times = {False: [], True: []}
    q_sum = ql_sum = None
    k0 = None
    for rep_ in range(2):
        for let in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for fi in range(len(nom.fields)):
                eng.run_dose(nom, fi, n_batches=0, sigma=False, let=let, fixed_point_bits=36)
                if let and rep_ == 1:
                    q, k = eng.last_tally(0)
                    ql, sh = eng.last_let(0)
                    k0 = k
                    q_sum = q.double() if q_sum is None else q_sum + q.double()
                    ql_sum = ql.double() * 2.0 ** sh if ql_sum is None else ql_sum + ql.double() * 2.0 ** sh
            torch.cuda.synchronize()
            times[let].append(time.perf_counter() - t0)
    roi = torch.from_numpy(I.head_structures(case, a.target_cc)).to(q_sum.device).reshape(q_sum.shape)
    out = {"s_plan_dose_without_let": min(times[False]), "s_plan_dose_with_let": min(times[True]),
           "let_cost": min(times[True]) / min(times[False]) - 1.0, "fixed_point_bits": k0}
    for name, bit in (("target", 1), ("oar", 2)):
        m = (roi & bit) != 0
        out[f"let_d_kev_per_um_{name}"] = float(ql_sum[m].sum() / q_sum[m].sum())
    progress(f"LET tally: plan dose {out['s_plan_dose_without_let']:.3f} s -> {out['s_plan_dose_with_let']:.3f} s "
             f"(+{100 * out['let_cost']:.1f} %); LET_d target {out['let_d_kev_per_um_target']:.2f}, "
             f"organ {out['let_d_kev_per_um_oar']:.2f} keV/um")
    return out


def resolution_study(a, np):
    """Dose-grid resolution (the paper's 2 mm vs 1 mm observation, Discussion;
    IM memory): the head case's spots, fields and scenarios
    on CT grids of 1x1x2, 1x1x1 and 2x2x2 mm over the same 256x256x320 mm
    volume, the same VPs per spot everywhere.  Per grid: seconds per
    13-scenario IM (one warm-up, one timed), non-zeros, CSR bytes, U of the
    uniform-weight plan dose; then the plan dose (4x the VPs) of the coarse
    grids, read as constant over each coarse voxel and trilinear between the
    coarse voxels' centres, against the 1 mm dose: global gamma 2 %/2 mm and
    1 %/1 mm (10 % threshold) over the bounding box of the 10 % region, the
    fraction of voxels within 2 % of the maximum in the high-dose (>= 50 %)
    and 10-50 % regions, the high-dose mean ratio.  Prints one JSON line (not
    the bench line)."""
    import torch
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gamma import gamma_pass_rate
    base = I.config4(a.target_cc, int(a.histories_per_spot))
    ext = (256.0, 256.0, 320.0)
    grids = {"1x1x2": (1.0, 1.0, 2.0), "1x1x1": (1.0, 1.0, 1.0), "2x2x2": (2.0, 2.0, 2.0)}
    eng = V.Engine(0)
    out, doses = {}, {}
    for name, sp in grids.items():
        shape = tuple(int(round(e / h)) for e, h in zip(ext, sp))
        case = I.Case(f"head_{name}", I.head_ct(0, shape=shape, spacing=sp), base.fields, base.scenarios,
                      seed=base.seed, physics=base.physics)
        eng.load_case(case)
        for rep_ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp, col, val, _, _ = eng.run_csr(case, device_out=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            nnz = int(col.numel())
            del rp, col, val
        u = plan_uncertainty(eng, case, I, V, np)
        d, _ = plan_dose(eng, case, I, mult=4)
        doses[name] = d.cpu().numpy().reshape(shape[::-1])
        out[name] = {"shape": shape, "s_per_13_scenario_im": dt, "nnz": nnz, "csr_gb_int32_fp32": 8e-9 * nnz,
                     "plan_dose_uncertainty": u}
        progress(f"resolution {name}: {dt:.2f} s per IM, nnz {nnz}, U {u:.4f}")
    eng.close()
    ref = doses["1x1x1"]
    m = np.argwhere(ref >= 0.1 * ref.max())
    lo = np.maximum(m.min(0) - 3, 0)
    hi = np.minimum(m.max(0) + 4, ref.shape)
    box = tuple(slice(l, h) for l, h in zip(lo, hi))
    from scipy.ndimage import map_coordinates
    rb = ref[box]
    hi_region = rb >= 0.5 * ref.max()
    mid_region = (rb >= 0.1 * ref.max()) & ~hi_region
    for name in ("1x1x2", "2x2x2"):
        fx, fy, fz = (int(round(h)) for h in grids[name])
        res = {}
        # the coarse dose read as constant over each coarse voxel, and
        # trilinear between the coarse voxels' centres
        zz, yy, xx = np.meshgrid(*[np.arange(l, h) for l, h in zip(lo, hi)], indexing="ij")
        cz, cy, cx = (zz + 0.5) / fz - 0.5, (yy + 0.5) / fy - 0.5, (xx + 0.5) / fx - 0.5
        evs = {"constant": np.repeat(np.repeat(np.repeat(doses[name], fz, 0), fy, 1), fx, 2)[box],
               "trilinear": map_coordinates(doses[name].astype(np.float64), [cz, cy, cx], order=1, mode="nearest")}
        for how, ev in evs.items():
            g22 = gamma_pass_rate(rb, ev, (1.0, 1.0, 1.0), 0.02, 2.0)
            g11 = gamma_pass_rate(rb, ev, (1.0, 1.0, 1.0), 0.01, 1.0)
            d = np.abs(ev - rb) / ref.max()
            res[how] = {"gamma_2pct_2mm": g22, "gamma_1pct_1mm": g11,
                        "within_2pct_of_max_high_dose": float((d[hi_region] <= 0.02).mean()),
                        "within_2pct_of_max_10_50pct": float((d[mid_region] <= 0.02).mean()),
                        "high_dose_mean_ratio": float(ev[hi_region].mean() / rb[hi_region].mean())}
            progress(f"{name} ({how}) vs 1x1x1: gamma 2%/2mm {g22:.4f}, 1%/1mm {g11:.4f}, "
                     f"|dD| <= 2% of max: high {res[how]['within_2pct_of_max_high_dose']:.4f} "
                     f"10-50% {res[how]['within_2pct_of_max_10_50pct']:.4f}, "
                     f"high-dose mean ratio {res[how]['high_dose_mean_ratio']:.4f}")
        out[name]["vs_1mm"] = res
    print(json.dumps({"study": "dose-grid resolution of the head IM", "histories_per_spot": a.histories_per_spot,
                      "grids": out}), flush=True)


def cpu_baseline(case, seconds, np):
    """The oracle on a bounded sample of the same workload: nominal scenario,
    first field, every 10th spot, the same VP count per spot, grown until
    one run takes at least 0.6 x `seconds`.  Returns histories/s."""
    import oracle
    from paper_2307_01416_amd import inputs as I
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    f = case.fields[0]
    sub = I.Field(beam=f.beam, spots=f.spots[::10].copy(), polygon=f.polygon, block=f.block, rs=f.rs)
    probe = I.Case("probe", case.geometry, [sub], [I.Scenario()], seed=case.seed, physics=case.physics)
    per_spot = 200
    while True:
        sub.spots["n_histories"] = per_spot
        t0 = time.perf_counter()
        oracle.run_tally(probe, threads=threads)
        dt = time.perf_counter() - t0
        n = int(np.sum(sub.spots["n_histories"]))
        if dt >= 0.6 * seconds or per_spot >= 10_000_000:
            break
        per_spot = int(per_spot * min(50.0, max(2.0, 1.1 * seconds / max(dt, 1e-3))))
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"nominal scenario, field 1, {len(sub.spots)} of {len(f.spots)} spots x {per_spot} VPs "
                      f"({n} VPs, full physics, {dt:.1f} s on {cpu})"}


def oracle_suite(np):
    """The oracle beside the GPU on the small workloads: config 1 in full,
    two config-2 cases in full (all host threads), and single-thread rates
    on bounded samples; one JSON line per case."""
    import oracle
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    import torch
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    eng = V.Engine(0)
    cases = [("config1 water 100 MeV", I.config1(100_000)),
             ("config2 10 mm opening + RS", I.config2(10.0, True)),
             ("config2 40 mm opening, no RS", I.config2(40.0, False))]
    for name, c in cases:
        n = int(np.sum(c.fields[0].spots["n_histories"]))
        eng.load_case(c)
        eng.run_dose(c, 0, n_batches=0, sigma=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.run_dose(c, 0, n_batches=0, sigma=False)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        progress(f"{name}: GPU {n} VPs in {t_gpu:.3f} s; oracle on {threads} threads ...")
        t0 = time.perf_counter()
        oracle.run_tally(c, threads=threads)
        t_all = time.perf_counter() - t0
        # single thread on a sample sized for about 4 s (ideal scaling assumed)
        sub = I.Field(beam=c.fields[0].beam, spots=c.fields[0].spots.copy(), polygon=c.fields[0].polygon,
                      block=c.fields[0].block, rs=c.fields[0].rs)
        frac = min(1.0, 4.0 / max(t_all * threads, 1e-3))
        sub.spots["n_histories"] = np.maximum(1, (sub.spots["n_histories"] * frac).astype(np.uint32))
        probe = I.Case("probe", c.geometry, [sub], c.scenarios, seed=c.seed, physics=c.physics)
        n1 = int(np.sum(sub.spots["n_histories"]))
        t0 = time.perf_counter()
        oracle.run_tally(probe, threads=1)
        t_one = time.perf_counter() - t0
        print(json.dumps({"case": name, "histories": n, "gpu_s": t_gpu, "gpu_histories_per_s": n / t_gpu,
                          "oracle_threads": threads, "oracle_s": t_all, "oracle_histories_per_s": n / t_all,
                          "oracle_1thread_sample": n1, "oracle_1thread_s": t_one,
                          "oracle_1thread_histories_per_s": n1 / t_one,
                          "gpu_over_oracle": (n / t_gpu) / (n / t_all)}), flush=True)
    eng.close()


def main():
    a = parse()
    if a.oracle_suite:
        import numpy as np
        oracle_suite(np)
        return
    if a.resolution_study:
        import numpy as np
        resolution_study(a, np)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V

    if a.copy_calibration:
        copy_calibration()
    progress("building the synthetic head case ...")
    H = a.histories_per_spot
    case = I.config4(a.target_cc, int(H), layer_apertures=a.layer_apertures,
                     n_vertices=32 if a.layer_apertures else 128)
    if a.divergent > 0.0:
        for f in case.fields:
            f.vsad_mm = a.divergent
            f.block.focus_mm = a.divergent
    eng = V.Engine(0)
    eng.load_case(case)

    # scale the history counts until the nominal plan dose reaches U <= 0.5 %
    u = None if a.no_scale else plan_uncertainty(eng, case, I, V, np)
    if u is not None:
        progress(f"U at {H:.0f} VPs/spot (mean): {u:.4f}")
    if u is not None and u > TARGET_U:
        f = (u / TARGET_U) ** 2 * 1.05
        for fl in case.fields:
            fl.spots["n_histories"] = np.ceil(fl.spots["n_histories"] * f).astype(np.uint32)
        H *= f
        u = plan_uncertainty(eng, case, I, V, np)
        progress(f"U at {H:.0f} VPs/spot (mean): {u:.4f}")
    eng.load_case(case)
    shape = dict(hist_per_lane=0, grid_blocks=0, block_threads=0)
    if a.shape:
        h, b, t = (int(v) for v in a.shape.split(","))
        shape = dict(hist_per_lane=h, grid_blocks=b, block_threads=t)
    elif not a.no_autotune:
        # launch shape of the work queue (hist_per_lane, workgroups, threads)
        # from each field's spots; kept on the context (histories per lane
        # per field, used by the epochs of that field)
        picks = []
        for fi, fl in enumerate(case.fields):
            best = V.vpmc_autotune(eng.ctx, fi, V.spot_array(fl.spots), len(fl.spots),
                                   V.scenario_array([I.Scenario()]),
                                   V.make_opts(seed=case.seed, physics=case.physics, output=V.OUT_CSR),
                                   sample_histories=int(2e7))
            picks.append(best.hist_per_lane)
        progress(f"autotune: hist_per_lane per field={picks} grid_blocks={best.grid_blocks} "
                 f"threads={best.block_threads}")
    shape_used = dict(shape)
    if not a.shape and not a.no_autotune:
        shape_used = dict(hist_per_lane_per_field=picks, grid_blocks=best.grid_blocks,
                          block_threads=best.block_threads)
    n_rows = len(case.scenarios) * sum(len(fl.spots) for fl in case.fields)
    n_hist_step = len(case.scenarios) * sum(int(np.sum(fl.spots["n_histories"])) for fl in case.fields)

    def step():
        # the influence matrices end as device-resident CSR (int32 voxel,
        # FP32 Gy per unit weight); they are dropped after the step
        rp, col, val, _, _ = eng.run_csr(case, graph=a.graph, device_out=True, **shape)
        st = V.vpmc_last_stats(eng.ctx)
        nnz = int(col.numel())
        del col, val
        return nnz, st

    for w in range(a.warmup):
        nnz, st = step()
        progress(f"warmup {w}: {st['total_ms']:.0f} ms, nnz {nnz}")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(a.steps):
        nnz, st = step()
        stats.append(st)
        progress(f"step {k}: {time.perf_counter() - t0:.2f} s elapsed")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    hist = sum(s["histories"] for s in stats)
    steps_total = sum(s["steps"] for s in stats)
    transport_s = sum(s["transport_ms"] for s in stats) * 1e-3
    launches = sum(s["launches"] for s in stats)
    assert hist == n_hist_step * a.steps, (hist, n_hist_step * a.steps)
    achieved = ALG_OPS_PER_STEP * steps_total / transport_s
    out = {
        "metric": "VP histories/s; s per 13-scenario influence matrix at 0.5% dose uncertainty",
        "value": hist / dt,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+int64",
        "data": "synthetic",
        "s_per_13_scenario_im": dt / a.steps,
        "config": {"workload": f"synthetic head CT 256x256x160 @1x1x2 mm, {a.target_cc} cc target, 3 coplanar "
                               f"fields with brass aperture (+5 mm) and 45 mm WET PMMA range shifter, "
                               f"13 robust scenarios, per-spot CSR influence matrices"
                               + (", energy-layer-specific apertures (one field per layer)" if a.layer_apertures else "")
                               + (f", virtual source and divergent block focused {a.divergent:.0f} mm upstream"
                                  if a.divergent > 0.0 else ""),
                   "rows": n_rows, "histories_per_step": n_hist_step,
                   "mean_histories_per_spot": float(H), "plan_dose_uncertainty": u, "nnz": nnz,
                   "csr_gb": nnz * 8 / 1e9, "graph": bool(a.graph), "launch_shape": shape_used},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_PEAK_FLOPS / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_FLOPS, "traffic": measured_traffic(),
                     "kernel": "queue_kernel", "avg_launch_ms": 1e3 * transport_s / max(1, launches),
                     "steps_per_s": steps_total / transport_s, "alg_ops_per_step": ALG_OPS_PER_STEP,
                     "lane_op_peak": VALU_PEAK_OPS / 1e12, "frac_of_lane_op_peak": achieved / VALU_PEAK_OPS},
        "transport_fraction_of_wall": transport_s / dt,
        "paper_context": "VPMC 41.6 s for 13 influence matrices (mean of 3 patients, 1-2 fields), "
                         "EPYC 7543 + 4x A100",
        "device": torch.cuda.get_device_name(0),
    }
    # what bounds the launch as built (from the committed counters of this
    # kernel source): its VALU instructions at the chip's issue rate, and its
    # memory-side int64 atomics (deposits outside the LDS row tile) at the
    # rate the atomic probe measures on the head grid
    rate = V.vpmc_atomic_rate(eng.ctx, case.geometry.shape, 1 << 28)
    t_launch = transport_s / max(1, launches)
    insts = measured_traffic(key="valu_insts_per_launch")
    atomics = measured_traffic(key="memside_atomics_per_launch")
    floor = {"atomic_rate_per_s": rate, "t_launch_ms": 1e3 * t_launch,
             "valu_insts_per_launch": insts, "memside_atomics_per_launch": atomics}
    if insts is not None and atomics is not None:
        t_issue, t_atom = insts / VALU_ISSUE_PEAK, atomics / rate
        floor.update({"t_valu_issue_ms": 1e3 * t_issue, "t_memside_atomics_ms": 1e3 * t_atom,
                      "bound": "valu_issue" if t_issue >= t_atom else "memside_atomics",
                      "frac": max(t_issue, t_atom) / t_launch,
                      "valu_lane_slots_per_step": insts * 64 * max(1, launches) / steps_total})
        progress(f"launch {1e3 * t_launch:.2f} ms: VALU issue floor {1e3 * t_issue:.2f} ms, memory-side atomics "
                 f"{1e3 * t_atom:.2f} ms")
    out["issue_floor"] = floor
    if not a.no_per_spot:
        ps = per_spot_baseline(eng, case, I, V, np)
        ps["batched_speedup"] = ps["s_per_13_scenario_im_extrapolated"] / (dt / a.steps)
        out["per_spot_baseline"] = ps
    if not a.no_surrogate:
        out["surrogate"] = surrogate_comparison(eng, case, I, V, np, a, shape, dt / a.steps,
                                                steps_total / a.steps)
        if "per_spot_baseline" in out:
            out["surrogate"]["batched_surrogate_speedup_vs_per_spot"] = (
                out["per_spot_baseline"]["s_per_13_scenario_im_extrapolated"] / out["surrogate"]["s_per_13_scenario_im"])
    if not a.no_optimize:
        out["optimizer"] = optimizer_measure(eng, case, I, V, np, torch, a, shape)
    if a.dynamic_spacing:
        out["dynamic_spacing"] = dynamic_spacing_measure(eng, case, I, V, np, torch, a, shape)
    if a.let:
        out["let"] = let_measure(eng, case, I, V, np, torch, a)
    if not a.no_cpu_baseline:
        progress("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds, np)
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
