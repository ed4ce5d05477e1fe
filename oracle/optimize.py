"""FP64 reference of the robust spot-weight optimisation on the influence
matrices (the plan optimisation the paper's workflow runs on the
13-scenario influence matrices, Methods E).  TEST INFRASTRUCTURE ONLY, like
the rest of this package.

Objective (reading: scenario-averaged "composite" objective, with the usual
quadratic prescription and maximum-dose penalties):
    F(x) = 1/S sum_s [ wT sum_{v in T} (D_s(v) - dp)^2
                       + wO sum_{v in O} max(0, D_s(v) - dmax)^2 ],
    D_s = A_s^T x,  x >= 0 (one weight per spot, shared by the scenarios),
where A_s[j, v] is the dose in voxel v per unit weight of spot j in scenario
s.  Gradient: 2/S sum_s A_s r_s with r_s = wT (D_s - dp) on T + wO max(0,
D_s - dmax) on O.  Solver: FISTA (Beck and Teboulle 2009) with the
projection onto x >= 0 and the fixed step 1/L, L = 1.05 x the largest
eigenvalue of 2/S sum_s A_s M A_s^T (M = wT on T + wO on O) from n_power
power iterations started at the all-ones vector.  Reading for the
degenerate case (no curvature: all of M A_s^T vanishes): the eigenvalue is
0, the power vector stays as it is and each step is the projection alone."""
from __future__ import annotations

import numpy as np


def objective_grad(A, x, tmask, omask, dp, wT, dmax, wO):
    """(F, grad) at x; A: list of scipy.sparse matrices [n_spots, nvox] per scenario."""
    S = len(A)
    F = 0.0
    g = np.zeros_like(x)
    for As in A:
        D = As.T @ x
        r = np.zeros_like(D)
        dt = D[tmask] - dp
        r[tmask] += wT * dt
        F += wT * np.dot(dt, dt)
        do = np.maximum(0.0, D[omask] - dmax)
        r[omask] += wO * do
        F += wO * np.dot(do, do)
        g += As @ r
    return F / S, 2.0 * g / S


def lipschitz(A, tmask, omask, wT, wO, n_power=20):
    S = len(A)
    m = wT * tmask.astype(np.float64) + wO * omask.astype(np.float64)
    z = np.ones(A[0].shape[0])
    lam = 0.0
    for _ in range(n_power):
        y = np.zeros_like(z)
        for As in A:
            y += As @ (m * (As.T @ z))
        y *= 2.0 / S
        ny_ = float(np.linalg.norm(y))
        lam = ny_ / float(np.linalg.norm(z))
        if ny_ > 0.0:
            z = y / ny_
    return 1.05 * lam


def fista(A, x0, tmask, omask, dp, wT, dmax, wO, iters, n_power=20):
    """Returns (x, objective at each extrapolated point y_k then at the final
    x [iters + 1], L)."""
    L = lipschitz(A, tmask, omask, wT, wO, n_power)
    x = np.maximum(np.asarray(x0, np.float64), 0.0)
    y = x.copy()
    t = 1.0
    hist = []
    for _ in range(iters):
        F, g = objective_grad(A, y, tmask, omask, dp, wT, dmax, wO)
        hist.append(F)
        xn = np.maximum(0.0, y - g / L if L > 0.0 else y)
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        y = xn + ((t - 1.0) / tn) * (xn - x)
        x, t = xn, tn
    hist.append(objective_grad(A, x, tmask, omask, dp, wT, dmax, wO)[0])
    return x, np.array(hist), L


def matrices_from_csr(row_ptr, col, val, n_scen, n_spots, nvox, row_stride=0, row_offset=0):
    """Scenario matrices A_s [n_spots, nvox] (FP64) from CSR rows
    s*row_stride + row_offset + j."""
    import scipy.sparse as sp
    stride = row_stride or n_spots
    A = []
    for s in range(n_scen):
        r0 = s * stride + row_offset
        rp = np.asarray(row_ptr[r0: r0 + n_spots + 1], np.int64)
        lo, hi = int(rp[0]), int(rp[-1])
        A.append(sp.csr_matrix((np.asarray(val[lo:hi], np.float64), np.asarray(col[lo:hi], np.int64), rp - lo),
                               shape=(n_spots, nvox)))
    return A
