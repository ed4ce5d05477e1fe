"""Write the FP64 oracle's full-physics doses of the head parity cases.

Calls only the oracle and the seeded inputs (``tests/head_cases.py``):
    python tests/golden/make_head_physics.py [case names ...] [--threads N]

For each case the oracle transports ORACLE_HISTORIES VPs of the case's spot
in 16 batches (history h in batch h mod 16) and the file keeps, for the
non-air voxels whose dose is at least 5 % of the non-air maximum, the dose
and its batch standard error (FP32, Gy per VP), the per-batch doses of the
voxels at or above 25 % (for the error of a regional mean), the non-air
maximum, the uncertainty U (mean sigma/D over non-air voxels >= 50 % of the
maximum), the energy ledger, the hash of the inputs and a fingerprint of the
oracle's results (head_cases.oracle_fingerprint) so that a stale file is
detected.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
import head_cases as H  # noqa: E402


def make(name: str, threads: int) -> None:
    c = H.case(name, H.ORACLE_HISTORIES, H.ORACLE_SEED)
    t0 = time.time()
    r = oracle.dose(c, n_batches=H.N_BATCHES, keep_batches=True, threads=threads)
    dt = time.time() - t0
    body = H.body_mask(c)
    d = r["dose_gy"]
    dmax = float(np.max(np.where(body, d, 0.0)))
    keep = body & (d >= H.STORE_FRACTION * dmax)
    idx = np.flatnonzero(keep.ravel())
    bkeep = body & (d >= H.BATCH_FRACTION * dmax)
    bidx = np.flatnonzero(bkeep.ravel())
    hi = body & (d >= 0.5 * dmax)
    u = float(np.mean(r["sigma_gy"][hi] / d[hi]))
    np.savez_compressed(
        H.golden_file(name),
        idx=idx.astype(np.int32),
        dose_gy=d.ravel()[idx].astype(np.float32),
        sigma_gy=r["sigma_gy"].ravel()[idx].astype(np.float32),
        batch_idx=bidx.astype(np.int32),
        batch_dose_gy=np.stack([b.ravel()[bidx] for b in r["batch_dose_gy"]]).astype(np.float32),
        body_max_gy=np.float64(dmax),
        uncertainty=np.float64(u),
        ledger_mev=r["ledger_mev"].astype(np.float64),
        n_histories=np.int64(H.ORACLE_HISTORIES),
        seed=np.int64(H.ORACLE_SEED),
        n_batches=np.int64(H.N_BATCHES),
        input_hash=np.array(H.input_hash(c)),
        oracle_fingerprint=np.array(H.oracle_fingerprint()),
        seconds=np.float64(dt),
        threads=np.int64(threads),
    )
    print(f"{name}: {H.ORACLE_HISTORIES} VPs in {dt:.0f} s ({H.ORACLE_HISTORIES / dt:.3e} VPs/s), U {u:.4f}, "
          f"stored {idx.size} voxels, batch voxels {bidx.size}", flush=True)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for name in (a.names or list(H.CASES)):
        make(name, a.threads)


if __name__ == "__main__":
    main()
