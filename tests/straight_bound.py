"""Per-voxel allowance for the straight-mode parity test (test tooling).

In straight mode (no straggling, scattering or nuclear events) a history's
path is fixed by its start position, which the GPU computes in FP32 and the
oracle in FP64.  A history that starts within BAND_MM of a lateral voxel
boundary, of an edge of the aperture polygon or of the range shifter's rim
may therefore take the other side of it on the GPU.  For each such history the
oracle transports it twice more with its start moved across each of those
boundaries (mirror image, the rest of the history unchanged: straight mode
draws no random numbers after the source); the largest difference between the
original and a moved copy's per-voxel deposits bounds what the FP32 rounding
of that history's start can change in each voxel.  The parity test then
demands, in every voxel,

    |D_gpu - D_or| <= 1e-5 D_or + allowance + 1e-11 D_max,

so nothing is excluded, and it checks that the allowances add up to at most
0.2 % of the dose (a history whose start flips to the neighbouring column
moves at most twice its energy; about 2e-4 of the histories start within the
band of a 1 mm voxel boundary along the two lateral axes).

BAND_MM: an FP32 start position is a handful of roundings of coordinates up
to ~260 mm (the spot's Gaussian offset, the beam-to-CT transform, the
subtraction of the grid origin), each at most half an ulp of 256, 1.5e-5 mm;
three of them stay below 5e-5 mm.
"""
from __future__ import annotations

import copy
import itertools
import math

import numpy as np

BAND_MM = 5e-5


def source_xy_fp64(orc, case, field_index, spot_index, n):
    """FP64 beam's-eye-view start positions of the first n histories of a spot
    (Box-Muller on the first two words of Philox block 0; parallel beams)."""
    f = case.fields[field_index]
    sp = f.spots[spot_index]
    key = [case.seed & 0xFFFFFFFF, ((case.seed >> 32) & 0xFFFFFFFF) ^ field_index]
    xs = np.empty(n)
    ys = np.empty(n)
    for h in range(n):
        w = orc.philox([0, h, spot_index, 0], key)
        u0, u1 = orc.uniform(int(w[0])), orc.uniform(int(w[1]))
        r = math.sqrt(-2.0 * math.log(u0))
        xs[h] = float(sp["x_mm"]) + float(sp["sigma_mm"]) * r * math.cos(2 * math.pi * u1)
        ys[h] = float(sp["y_mm"]) + float(sp["sigma_mm"]) * r * math.sin(2 * math.pi * u1)
    return xs, ys


def _polygon_nudges(poly, x, y):
    """Signed distance to the nearest edge and the move (dx, dy) that mirrors
    the point across that edge's line."""
    a = np.asarray(poly, np.float64)
    b = np.roll(a, -1, axis=0)
    best = (math.inf, 0.0, 0.0)
    for (ax_, ay_), (bx_, by_) in zip(a, b):
        ex, ey = bx_ - ax_, by_ - ay_
        L2 = ex * ex + ey * ey
        t = min(1.0, max(0.0, ((x - ax_) * ex + (y - ay_) * ey) / L2))
        px, py = ax_ + t * ex, ay_ + t * ey
        d = math.hypot(x - px, y - py)
        if d < best[0]:
            # unit normal of the edge, pointing from the line to the point
            nx_, ny_ = -ey / math.sqrt(L2), ex / math.sqrt(L2)
            s = (x - ax_) * nx_ + (y - ay_) * ny_
            best = (d, -2.0 * s * nx_, -2.0 * s * ny_)
    return best


def ambiguous_moves(orc, case, field_index=0, scenario_index=0, spots=None, band=BAND_MM):
    """{(spot, history): [(dx, dy), ...]} beam's-eye-view moves that put the
    history's start across each boundary it lies within `band` of."""
    g = case.geometry
    f = case.fields[field_index]
    ez = np.asarray(f.beam.ez, np.float64)
    ex = np.asarray(f.beam.ex, np.float64)
    ey = np.asarray(f.beam.ey, np.float64)
    ax = int(np.argmax(np.abs(ez)))
    assert abs(abs(ez[ax]) - 1.0) < 1e-12, "axis-aligned beams only"
    lat = [k for k in range(3) if k != ax]
    shift = np.asarray(case.scenarios[scenario_index].shift_mm, np.float64)
    origin = np.asarray(g.origin, np.float64) + shift
    sp = np.asarray(g.spacing, np.float64)
    out = {}
    for s in (range(len(f.spots)) if spots is None else spots):
        n = int(f.spots["n_histories"][s])
        x, y = source_xy_fp64(orc, case, field_index, s, n)
        p = np.asarray(f.beam.iso)[None, :] + x[:, None] * ex[None, :] + y[:, None] * ey[None, :]
        fr = (p - origin[None, :]) / sp[None, :]
        for h in range(n):
            moves = []
            for k in lat:
                d = (fr[h, k] - np.rint(fr[h, k])) * sp[k]
                if abs(d) < band:
                    # move the CT coordinate k by -2d (the BEV axes map onto CT axis k by ex[k], ey[k])
                    moves.append((-2.0 * d * ex[k], -2.0 * d * ey[k]))
            if f.polygon is not None and f.block is not None:
                d, dx, dy = _polygon_nudges(f.polygon, x[h], y[h])
                if d < band:
                    moves.append((dx, dy))
            if f.rs is not None:
                r = math.hypot(x[h], y[h])
                dr = r - 0.5 * f.rs.diameter_mm
                if abs(dr) < band and r > 0:
                    moves.append((-2.0 * dr * x[h] / r, -2.0 * dr * y[h] / r))
            if moves:
                out[(s, h)] = moves
    return out


def allowance(orc, case, field_index=0, scenario_index=0, spots=None, band=BAND_MM):
    """(allowance [nz, ny, nx] in tally units q * 2^-k = MeV * w/N, number of
    ambiguous histories)."""
    g = case.geometry
    nx, ny, nz = g.shape
    allow = np.zeros(nx * ny * nz)
    moves = ambiguous_moves(orc, case, field_index, scenario_index, spots, band)
    f = case.fields[field_index]
    for (s, h), mv in moves.items():
        _, _, base = orc.trace_history(case, s, h, field_index, scenario_index, want_grid=True)
        worst = np.zeros_like(base)
        for r in range(1, len(mv) + 1):
            for combo in itertools.combinations(mv, r):
                dx = sum(m[0] for m in combo)
                dy = sum(m[1] for m in combo)
                c2 = copy.copy(case)
                c2.fields = list(case.fields)
                f2 = copy.copy(f)
                f2.spots = f.spots.copy()
                f2.spots["x_mm"][s] = np.float32(float(f.spots["x_mm"][s]) + dx)
                f2.spots["y_mm"][s] = np.float32(float(f.spots["y_mm"][s]) + dy)
                c2.fields[field_index] = f2
                _, _, var = orc.trace_history(c2, s, h, field_index, scenario_index, want_grid=True)
                np.maximum(worst, np.abs(var - base), out=worst)
        w = float(f.spots["weight"][s]) / float(f.spots["n_histories"][s])
        allow += worst * w
    return allow.reshape(nz, ny, nx), len(moves)


def assert_straight_parity(q_gpu, k_gpu, q_or, k_or, allow=None, max_allow_share=2e-3, say=print):
    """1e-5 relative per voxel above 1e-6 of the maximum, 1e-11 of the maximum
    below, plus the per-voxel allowance of the ambiguous histories (and the
    fixed-point rounding of their deposits); the allowances may add up to at
    most max_allow_share of the dose."""
    a = q_gpu.astype(np.float64) * 2.0 ** -k_gpu
    b = q_or.astype(np.float64) * 2.0 ** -k_or
    dmax = b.max()
    assert dmax > 0
    al = np.zeros_like(b) if allow is None else allow
    share = al.sum() / b.sum()
    al = np.where(al > 0, al + 1e-3 * al + 2.0 ** -min(k_gpu, k_or) * 1e3, 0.0)
    hi = b > 1e-6 * dmax
    bound = np.where(hi, 1e-5 * b, 1e-11 * dmax) + al
    err = np.abs(a - b)
    strict = al == 0
    rel = err[hi & strict] / b[hi & strict]
    bad = err > bound
    say(f"  straight parity: {int(hi.sum())} voxels above 1e-6 of max, max rel {rel.max():.3e} over "
        f"{int((hi & strict).sum())} without allowance; {int((~strict).sum())} voxels with allowance "
        f"(its sum {share:.2e} of the dose, those voxels' dose share {b[~strict].sum() / b.sum():.2e}); "
        f"worst bound use {float(np.max(err / bound)):.3f}")
    assert not bad.any(), f"{int(bad.sum())} voxels outside the bound"
    assert share <= max_allow_share
