"""Throughput benchmark of the VP transport on one MI355X.

Workload (one step): the eight water-phantom cases with a 30 mm brass block
(openings 10/20/30/40 mm, each without and with a 45 mm WET PMMA range
shifter), water 200x200x300 at 1 mm, spots on a 2.5 mm grid over the
opening + 5 mm, 1e7 virtual particles per case, full physics, 16 batches for
the per-voxel standard error.  Inputs are synthetic and resident on the GPU
before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operations per condensed-history step counted from the algorithm
# (Philox4x32-10 ~100 integer ops, uniform/normal conversion ~40, three table
# interpolations ~35, CSDA loss ~10, hinge rotation ~35, DDA ~15, nuclear
# test ~5, fixed-point tally ~5, position updates ~10)
ALG_OPS_PER_STEP = 255.0
# gfx950: 256 CUs x 64 FP32 lanes per clock x 2.4 GHz, single-issue VALU
VALU_PEAK_OPS = 256 * 64 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories-per-case", type=float, default=1e7)
    ap.add_argument("--batches", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=1.25e5, help="oracle histories per case")
    return ap.parse_args()


def cpu_baseline(n_per_case: int):
    import numpy as np
    import oracle
    from paper_2307_01416_amd import inputs as I
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    cases = I.config2_all(histories_per_case=n_per_case)
    t0 = time.perf_counter()
    n = 0
    for c in cases:
        oracle.run_tally(c, threads=threads)
        n += int(np.sum(c.fields[0].spots["n_histories"]))
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"8 water/brass cases x {n_per_case} VPs (full physics, single batch), {dt:.1f} s on {cpu}"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V

    H = int(a.histories_per_case)
    cases = I.config2_all(histories_per_case=H)
    eng = V.Engine(0)
    eng.load_case(cases[0])
    n_hist_step = sum(int(np.sum(c.fields[0].spots["n_histories"])) for c in cases)

    def step(stats):
        for c in cases:
            for fi, f in enumerate(c.fields):
                V.vpmc_set_aperture(eng.ctx, fi, f)
            eng.run_dose(c, 0, n_batches=a.batches, sigma=True)
            stats.append(V.vpmc_last_stats(eng.ctx))

    def progress(msg):
        print(msg, file=sys.stderr, flush=True)

    for w in range(a.warmup):
        st = []
        step(st)
        progress(f"warmup {w}: {sum(s['transport_ms'] for s in st):.1f} ms transport")
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(stats)
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
        "config": {"workload": "water 200x200x300 @1 mm behind 30 mm brass block, openings 10/20/30/40 mm "
                               "x {no RS, 45 mm WET PMMA RS}; 2.5 mm spot grid; 1e7 VPs per case; "
                               "full physics; 16 batches",
                   "histories_per_step": n_hist_step, "cases": len(cases)},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "transport_kernel", "avg_launch_ms": 1e3 * transport_s / launches,
                     "steps_per_s": steps_total / transport_s},
        "transport_fraction_of_wall": transport_s / dt,
        "device": torch.cuda.get_device_name(0),
    }
    if not a.no_cpu_baseline:
        progress("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(int(a.cpu_sample))
    eng.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
