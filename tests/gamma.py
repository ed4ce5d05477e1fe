"""3D gamma pass rate (Low et al. 1998), global normalisation (test tooling).

Reading of the paper's "3D gamma analysis ... criterion of 2%/2 mm and a
threshold of 10%" (Methods D.1): dose difference relative to the reference
maximum; reference points below threshold * max are skipped; the evaluated
distribution is searched on a sub-grid of step <= DTA/4 by trilinear
interpolation.  Only the pass/fail decision is needed, so the search radius
is the DTA itself (a point farther than the DTA has gamma > 1).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _shift_trilinear(a: np.ndarray, off_vox) -> np.ndarray:
    """a evaluated at (index + off) with trilinear interpolation; outside the
    grid the value is NaN.  a is indexed [z, y, x]; off_vox is (ox, oy, oz)."""
    out = np.zeros_like(a, dtype=np.float64)
    valid = np.ones(a.shape, bool)
    fl = [math.floor(o) for o in off_vox]
    fr = [o - f for o, f in zip(off_vox, fl)]
    nz, ny, nx = a.shape
    for cx, cy, cz in itertools.product((0, 1), (0, 1), (0, 1)):
        w = (fr[0] if cx else 1 - fr[0]) * (fr[1] if cy else 1 - fr[1]) * (fr[2] if cz else 1 - fr[2])
        if w == 0.0:
            continue
        sx, sy, sz = fl[0] + cx, fl[1] + cy, fl[2] + cz
        src = np.full(a.shape, np.nan)
        zs = slice(max(0, -sz), min(nz, nz - sz))
        ys = slice(max(0, -sy), min(ny, ny - sy))
        xs = slice(max(0, -sx), min(nx, nx - sx))
        zd = slice(zs.start + sz, zs.stop + sz)
        yd = slice(ys.start + sy, ys.stop + sy)
        xd = slice(xs.start + sx, xs.stop + sx)
        src[zs, ys, xs] = a[zd, yd, xd]
        out += w * src
    return out


def gamma_pass_rate(ref: np.ndarray, ev: np.ndarray, spacing, dd: float, dta_mm: float,
                    threshold: float = 0.1, substep: float = 0.25) -> float:
    """Fraction of reference voxels >= threshold*max(ref) with gamma <= 1."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    dmax = ref.max()
    mask = ref >= threshold * dmax
    dcrit = dd * dmax
    best = np.full(ref.shape, np.inf)
    h = dta_mm * substep
    n = int(math.ceil(dta_mm / h))
    sx, sy, sz = spacing
    for i, j, k in itertools.product(range(-n, n + 1), repeat=3):
        r2 = (i * h) ** 2 + (j * h) ** 2 + (k * h) ** 2
        if r2 > dta_mm ** 2 + 1e-12:
            continue
        shifted = _shift_trilinear(ev, (i * h / sx, j * h / sy, k * h / sz))
        g2 = ((shifted - ref) / dcrit) ** 2 + r2 / dta_mm ** 2
        g2 = np.where(np.isnan(g2), np.inf, g2)
        np.minimum(best, g2, out=best)
    return float(np.mean(best[mask] <= 1.0 + 1e-12))


def gamma_bruteforce(ref, ev, spacing, dd, dta_mm, threshold=0.1, substep=0.25):
    """Same definition, one reference point at a time (tiny grids only)."""
    ref = np.asarray(ref, np.float64)
    ev = np.asarray(ev, np.float64)
    nz, ny, nx = ref.shape
    dmax = ref.max()
    h = dta_mm * substep
    n = int(math.ceil(dta_mm / h))
    sx, sy, sz = spacing

    def interp(x, y, z):
        if not (0 <= x <= nx - 1 and 0 <= y <= ny - 1 and 0 <= z <= nz - 1):
            return None
        x0, y0, z0 = min(int(x), nx - 2) if nx > 1 else 0, min(int(y), ny - 2) if ny > 1 else 0, \
            min(int(z), nz - 2) if nz > 1 else 0
        fx, fy, fz = x - x0, y - y0, z - z0
        val = 0.0
        for cx, cy, cz in itertools.product((0, 1), (0, 1), (0, 1)):
            w = (fx if cx else 1 - fx) * (fy if cy else 1 - fy) * (fz if cz else 1 - fz)
            if w:
                val += w * ev[z0 + cz, y0 + cy, x0 + cx]
        return val

    npass = ntot = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if ref[z, y, x] < threshold * dmax:
                    continue
                ntot += 1
                g = math.inf
                for i, j, k in itertools.product(range(-n, n + 1), repeat=3):
                    r2 = (i * h) ** 2 + (j * h) ** 2 + (k * h) ** 2
                    if r2 > dta_mm ** 2 + 1e-12:
                        continue
                    v = interp(x + i * h / sx, y + j * h / sy, z + k * h / sz)
                    if v is None:
                        continue
                    g = min(g, ((v - ref[z, y, x]) / (dd * dmax)) ** 2 + r2 / dta_mm ** 2)
                npass += g <= 1.0 + 1e-12
    return npass / ntot
