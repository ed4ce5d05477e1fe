"""Dynamic voxel spacing (coarser IM voxels for organs at risk,
Methods C) on the GPU against the FP64 reference, through the C ABI.  Inputs:
seeded pencil-beam-like rows (int64 fixed-point energies at k = 40, rows of
0 to ~10^3 entries, so runs cross the kernel's 64-entry windows), a seeded
head CT for the masses, the map of `dynamic_spacing_map` (target voxels
alone, organ voxels in pairs, the rest in fours along x).  Cells, row
pointers and int64 sums bit for bit; doses within 1e-6 relative (the GPU's
FP32 voxel densities against the reference's FP64)."""
import numpy as np
import pytest

import oracle as O
from oracle import cells as OC
from paper_2307_01416_amd import inputs as I
from test_gpu_parity import say

pytestmark = pytest.mark.gpu
K = 40


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01416_amd import vpmc as V
    P = I.opt_problem(seed=11, shape=(40, 36, 20), n_spots=30, n_scen=2)
    g = I.head_ct(3, shape=P.shape, spacing=(2.0, 2.0, 2.0))
    ctx = V.vpmc_create(0)
    V.vpmc_load_geometry(ctx, g)
    q = np.rint(P.val.astype(np.float64) * 2.0 ** K).astype(np.int64)
    _, rho = O.hu_lookup(g.hu)
    mass_g = rho.ravel() * (g.spacing[0] * g.spacing[1] * g.spacing[2] * 1e-3)
    yield V, ctx, P, g, q, mass_g
    V.vpmc_destroy(ctx)


def check(V, ctx, P, q, mass_g, cmap, n_cells, flags=0):
    import torch
    if flags:
        t = lambda a: torch.from_numpy(a).cuda()
        rp, cell, qo, val = V.vpmc_csr_cells(ctx, t(P.row_ptr), t(P.col), t(q), K, t(cmap), n_cells, flags)
        rp, cell, qo, val = (x.cpu().numpy() for x in (rp, cell, qo, val))
    else:
        rp, cell, qo, val = V.vpmc_csr_cells(ctx, P.row_ptr, P.col, q, K, cmap, n_cells)
    r_rp, r_cell, r_q, r_d = OC.cells_from_csr(P.row_ptr, P.col, q, K, cmap, mass_g, n_cells, O.lib().orc_mev_to_joule())
    assert np.array_equal(rp, r_rp) and np.array_equal(cell, r_cell) and np.array_equal(qo, r_q)
    np.testing.assert_allclose(val, r_d, rtol=1e-6)
    return rp


def test_cells_match_the_reference(setup):
    V, ctx, P, g, q, mass_g = setup
    cmap, n = I.dynamic_spacing_map(P.shape, P.roi, target=1, oar=2, other=4)
    rp = check(V, ctx, P, q, mass_g, cmap, n)
    say(f"dynamic spacing: {P.nvox} voxels -> {n} cells, entries {P.row_ptr[-1]} -> {rp[-1]}")
    assert rp[-1] < P.row_ptr[-1]
    check(V, ctx, P, q, mass_g, cmap, n, flags=V.DEVICE_PTRS)


@pytest.mark.parametrize("width", [1, 7, 40])
def test_uniform_runs(setup, width):
    """Runs of `width` voxels along x (1: the identity, 40: whole x rows)."""
    V, ctx, P, g, q, mass_g = setup
    nx = P.shape[0]
    x = np.arange(P.nvox) % nx
    start = (x % width == 0)
    cmap = (np.cumsum(start) - 1).astype(np.int32)
    check(V, ctx, P, q, mass_g, cmap, int(cmap[-1]) + 1)


def test_errors(setup):
    V, ctx, P, g, q, mass_g = setup
    cmap, n = I.dynamic_spacing_map(P.shape, P.roi)
    bad = P.col.copy()
    b = int(P.row_ptr[1] + 3)
    bad[b], bad[b + 1] = bad[b + 1], bad[b]           # not ascending inside a row
    import torch
    t = lambda a: torch.from_numpy(a).cuda()
    with pytest.raises(V.VpmcError) as ex:
        V.vpmc_csr_cells(ctx, t(P.row_ptr), t(bad), t(q), K, t(cmap), n, V.DEVICE_PTRS)
    assert ex.value.code == V.E_ARG
    m2 = cmap.copy()
    m2[5] = m2[4] + 2
    with pytest.raises(V.VpmcError) as ex:
        V.vpmc_csr_cells(ctx, P.row_ptr, P.col, q, K, m2, n)
    assert ex.value.code == V.E_ARG
