"""Per-voxel allowance for the straight-mode parity test (test tooling).

In straight mode (no straggling, scattering or nuclear events) a history's
path is fixed by its start position, which the GPU computes in FP32 and the
oracle in FP64.  A history that starts within BAND_MM of a lateral voxel
boundary, of an edge of the aperture polygon or of the range shifter's rim
may therefore take the other side of it on the GPU.  For each such history the
oracle transports it twice more with its start moved across each of those
boundaries (mirror image, the rest of the history unchanged: straight mode
draws no random numbers after the source; the move is applied to the FP64
start itself, oracle.move_allowance); the largest difference between the
original and a moved copy's per-voxel deposits bounds what the FP32 rounding
of that history's start can change in each voxel.  Tracks that are tilted
(virtual source, divergent block) cross boundaries at depths that depend on
the start continuously, so there every history is moved by BAND_MM along the
eight directions of the source plane's square (shift_allowance).  The parity
test then demands, in every voxel,

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


def _combined(mv):
    """Every non-empty combination of a history's moves, summed."""
    out = []
    for r in range(1, len(mv) + 1):
        for combo in itertools.combinations(mv, r):
            out.append((sum(m[0] for m in combo), sum(m[1] for m in combo)))
    return out


def allowance(orc, case, field_index=0, scenario_index=0, spots=None, band=BAND_MM, with_let=False):
    """(allowance [nz, ny, nx] in tally units q * 2^-k = MeV * w/N, number of
    ambiguous histories); with_let: also the allowance of the dose-averaged
    LET's numerator (deposit x LET, MeV keV/um * w/N) as a third item.  Each
    ambiguous history is transported with its start moved across every
    combination of the boundaries it lies near (oracle.move_allowance)."""
    moves = ambiguous_moves(orc, case, field_index, scenario_index, spots, band)
    entries = [(s, h, _combined(mv)) for (s, h), mv in sorted(moves.items())]
    res = orc.move_allowance(case, entries, field_index, scenario_index, want_let=with_let)
    if with_let:
        return res[0], len(moves), res[1]
    return res, len(moves)


SHIFTS = [(sx, sy) for sx in (-1, 0, 1) for sy in (-1, 0, 1) if sx or sy]


DIR_REL = 4e-7


def shift_allowance(orc, case, field_index=0, scenario_index=0, delta=BAND_MM, dir_rel=DIR_REL):
    """Allowance for tilted tracks (virtual source, divergent block): every
    history is moved by delta along the eight directions of the source
    plane's square (axes and diagonals).  A tilted track crosses lateral voxel
    boundaries and tilted walls at depths that move by delta / tilt when its
    start moves by delta, so no history is exempt; the moved copies bound
    what the FP32 start, whose error stays within delta on either axis, can
    move between voxels.

    With a virtual source the direction itself comes from the FP32 start
    through a sum of squares, a square root, a reciprocal and a product
    (relative error below dir_rel = 4e-7), and the path length per unit depth
    follows it: every depth-energy relation moves by at most dir_rel of the
    water-equivalent path, which is less than the CSDA range R(E).  Each
    history is therefore also transported with its energy moved by
    +-dir_rel R(E) S(E) (E the spot's highest energy, water), and that
    allowance is added to the lateral one."""
    f = case.fields[field_index]
    lat, ene = [], []
    for s in range(len(f.spots)):
        mv = [(delta * sx, delta * sy) for sx, sy in SHIFTS]
        n = int(f.spots["n_histories"][s])
        lat.extend((s, h, mv) for h in range(n))
        if f.vsad_mm > 0.0:
            e = float(f.spots["energy_mev"][s]) + 6.0 * float(f.spots["energy_sigma_mev"][s])
            de = dir_rel * float(orc.csda_range(0, e)) * float(orc.stopping_power(0, e))
            ene.extend((s, h, [(0.0, 0.0, de), (0.0, 0.0, -de)]) for h in range(n))
    allow = orc.move_allowance(case, lat, field_index, scenario_index)
    if ene:
        allow = allow + orc.move_allowance(case, ene, field_index, scenario_index)
    return allow


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
    say(f"  straight parity: {int(hi.sum())} voxels above 1e-6 of max, max rel {rel.max() if rel.size else 0.0:.3e} over "
        f"{int((hi & strict).sum())} without allowance; {int((~strict).sum())} voxels with allowance "
        f"(its sum {share:.2e} of the dose, those voxels' dose share {b[~strict].sum() / b.sum():.2e}); "
        f"worst bound use {float(np.max(err / bound)):.3f}")
    if bad.any():
        w = np.unravel_index(int(np.argmax(err / bound)), b.shape)
        say(f"  worst voxel {tuple(int(i) for i in w)}: gpu {a[w]:.9e} oracle {b[w]:.9e} "
            f"allowance {al[w]:.3e} bound {bound[w]:.3e}")
    assert not bad.any(), f"{int(bad.sum())} voxels outside the bound"
    assert share <= max_allow_share
