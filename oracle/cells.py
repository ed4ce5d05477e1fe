"""FP64 reference of dynamic voxel spacing for influence matrices (the
planning system stores organs at risk on coarser voxels to save IM
memory, Methods C).  TEST INFRASTRUCTURE ONLY, like the rest of this
package.

A cell is a run of consecutive voxels (linear index, x fastest) given by a
non-decreasing voxel -> cell map whose cells are all non-empty.  For every
row, the entries of one cell are merged: q_cell = sum of the int64 fixed-point
energies (exact), dose_cell = q_cell 2^-k MeV->J / (sum of the cell's voxel
masses): the cell's energy over its mass, i.e. the mass-weighted mean of its
voxels' doses."""
from __future__ import annotations

import numpy as np


def check_map(cell_of_voxel: np.ndarray, n_cells: int) -> None:
    m = np.asarray(cell_of_voxel, np.int64)
    d = np.diff(m)
    if m.size == 0 or m[0] != 0 or m[-1] != n_cells - 1 or np.any((d != 0) & (d != 1)):
        raise ValueError("cell map must run 0 .. n_cells-1 in steps of 0 or 1")


def cell_mass_g(cell_of_voxel, voxel_mass_g, n_cells):
    """Mass of each cell (g): the sum of its voxels' masses."""
    return np.bincount(np.asarray(cell_of_voxel, np.int64), weights=np.asarray(voxel_mass_g, np.float64).ravel(),
                       minlength=n_cells)


def cells_from_csr(row_ptr, col, q, k, cell_of_voxel, voxel_mass_g, n_cells, mev_to_joule):
    """(row_ptr, cell, q, dose_gy) of the merged rows; dose in Gy per unit
    weight, FP64."""
    check_map(cell_of_voxel, n_cells)
    cmap = np.asarray(cell_of_voxel, np.int64)
    mass = cell_mass_g(cmap, voxel_mass_g, n_cells)
    rows_c, rows_q = [], []
    out_ptr = [0]
    for r in range(len(row_ptr) - 1):
        b, e = int(row_ptr[r]), int(row_ptr[r + 1])
        cells = cmap[np.asarray(col[b:e], np.int64)]
        acc = {}
        for c, v in zip(cells.tolist(), np.asarray(q[b:e], np.int64).tolist()):
            acc[c] = acc.get(c, 0) + v
        ks = sorted(acc)
        rows_c.append(np.array(ks, np.int64))
        rows_q.append(np.array([acc[c] for c in ks], np.int64))
        out_ptr.append(out_ptr[-1] + len(ks))
    cell = np.concatenate(rows_c) if rows_c else np.zeros(0, np.int64)
    qc = np.concatenate(rows_q) if rows_q else np.zeros(0, np.int64)
    dose = qc.astype(np.float64) * 2.0 ** (-k) * mev_to_joule / (mass[cell] * 1e-3)
    return np.array(out_ptr, np.int64), cell, qc, dose
