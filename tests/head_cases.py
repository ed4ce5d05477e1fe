"""Full-physics parity cases on the synthetic head CT (test tooling).

One pencil-beam spot of one of the three coplanar head fields (gantry 90,
180, 270 degrees; each with its brass aperture and range shifter, Methods D.3)
under one of the 13 robust scenarios (Methods E: setup shift and range
scaling).  Spots are taken from the most populated energy layer: the one on
the central axis, or the one centred on the aperture's edge (half of its
beam hits the brass), or the central spot of the most distal layer.

The FP64 oracle's doses of these cases are expensive at the history counts
the 0.25 % uncertainty target asks for (about 4e7 VPs per spot), so they are
written once by ``tests/golden/make_head_physics.py`` (which calls only the
oracle and these seeded inputs) and stored with the hash of the inputs and a
fingerprint of the oracle's results; a CPU test checks that both are still
current.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

from paper_2307_01416_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")

# name -> (field index 0/1/2 = gantry 90/180/270, scenario index in
#          inputs.scenarios_13(), spot kind)
CASES = {
    "g90_nominal_central": (0, 0, "central"),
    "g180_nominal_central": (1, 0, "central"),
    "g270_nominal_central": (2, 0, "central"),
    "g90_xplus_r1035_edge": (0, 1, "edge"),      # +3 mm along x, range x1.035
    "g180_yminus_r0965_edge": (1, 8, "edge"),    # -3 mm along y, range x0.965
    "g270_zplus_r1035_distal": (2, 9, "distal"),  # +3 mm along z, range x1.035
}

ORACLE_HISTORIES = 40_000_000
ORACLE_SEED = 20_231_001
GPU_SEED = 0
N_BATCHES = 16
STORE_FRACTION = 0.05     # oracle voxels stored: dose >= 5 % of the body maximum
BATCH_FRACTION = 0.25     # per-batch doses stored for voxels >= 25 % of it
AIR_HU = -900             # below: air (HU calibration breakpoint), excluded from comparisons


def _pick_spot(spots: np.ndarray, kind: str) -> int:
    e = spots["energy_mev"]
    vals, counts = np.unique(e, return_counts=True)
    layer = vals[np.argmax(counts)] if kind != "distal" else vals.max()
    sel = np.nonzero(e == layer)[0]
    x, y = spots["x_mm"][sel].astype(np.float64), spots["y_mm"][sel].astype(np.float64)
    if kind == "edge":
        # outermost spot on the +x half-axis of the beam's-eye view: it sits
        # on the opening's edge (the layer's disk and the opening share the
        # 5 mm margin)
        on_axis = np.abs(y) < 1e-6
        cand = np.nonzero(on_axis)[0]
        return int(sel[cand[np.argmax(x[cand])]])
    return int(sel[np.argmin(np.hypot(x, y))])


def case(name: str, n_histories: int, seed: int):
    """The single-field, single-spot, single-scenario head case of ``name``."""
    fi, si, kind = CASES[name]
    full = I.config3(8.0, 1)
    f = full.fields[fi]
    s = _pick_spot(f.spots, kind)
    f.spots = f.spots[s:s + 1].copy()
    f.spots["n_histories"] = n_histories
    f.spots["weight"] = 1.0
    scen = I.scenarios_13()[si]
    return I.Case(f"head_{name}", full.geometry, [f], [scen], seed=seed, physics=I.PHYS_ALL,
                  n_batches=N_BATCHES)


def body_mask(c) -> np.ndarray:
    """Non-air voxels [nz, ny, nx] (HU >= -900)."""
    return c.geometry.hu >= AIR_HU


def input_hash(c) -> str:
    """Hash of everything that defines the case except the history count and
    the seed: CT numbers, grid, beam, aperture, range shifter, spot, scenario."""
    h = hashlib.sha256()
    g = c.geometry
    h.update(np.ascontiguousarray(g.hu).tobytes())
    h.update(np.asarray(g.shape + g.spacing + g.origin, np.float64).tobytes())
    f = c.fields[0]
    b = f.beam
    h.update(np.asarray(b.iso + b.ex + b.ey + b.ez, np.float64).tobytes())
    h.update(np.ascontiguousarray(f.polygon).tobytes())
    h.update(np.asarray([f.block.thickness_mm, f.block.density_gcc, f.block.downstream_mm, f.block.focus_mm,
                         f.rs.wet_mm, f.rs.diameter_mm, f.rs.downstream_mm], np.float64).tobytes())
    sp = f.spots.copy()
    sp["n_histories"] = 0
    h.update(sp.tobytes())
    s = c.scenarios[0]
    h.update(np.asarray(s.shift_mm + (s.range_scale,), np.float64).tobytes())
    return h.hexdigest()


def oracle_fingerprint() -> str:
    """What the oracle computes, not how its source reads: the SHA-256 of the
    int64 tally and ledgers of 3000 full-physics histories of the aperture-edge
    head case (range shifter, brass, air, bone and brain, a shifted and
    range-scaled scenario) on one thread.  Any change of the transport's
    arithmetic changes these bits; edits that leave it alone do not."""
    import oracle
    c = case("g90_xplus_r1035_edge", 3000, 7)
    q, led, k = oracle.run_tally(c, threads=1)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(q).tobytes())
    h.update(np.ascontiguousarray(led).tobytes())
    h.update(np.int64(k).tobytes())
    return h.hexdigest()


def golden_file(name: str) -> str:
    return os.path.join(GOLDEN_DIR, f"head_physics_{name}.npz")


def load_golden(name: str, shape_zyx):
    """Oracle dose, sigma and per-batch doses of a stored case as dense
    [nz, ny, nx] FP64 grids (zero outside the stored voxels)."""
    z = np.load(golden_file(name), allow_pickle=False)
    n = int(np.prod(shape_zyx))
    dose = np.zeros(n)
    sigma = np.zeros(n)
    idx = z["idx"].astype(np.int64)
    dose[idx] = z["dose_gy"]
    sigma[idx] = z["sigma_gy"]
    out = {k: z[k] for k in z.files}
    out["dose"] = dose.reshape(shape_zyx)
    out["sigma"] = sigma.reshape(shape_zyx)
    return out
