"""Pins of the FP64 reference optimiser, no GPU: gradient by central
differences; with only a prescription term on every voxel the problem is
non-negative least squares, whose optimum scipy.optimize.nnls gives; the
power-iteration Lipschitz bound against the exact largest eigenvalue."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import nnls

from oracle import optimize as O


def _problem(seed=0, S=3, n=12, nvox=60, density=0.3):
    rng = np.random.default_rng(seed)
    A = [sp.random(n, nvox, density=density, random_state=rng, format="csr") * 0.01 for _ in range(S)]
    tmask = np.zeros(nvox, bool)
    tmask[10:30] = True
    omask = np.zeros(nvox, bool)
    omask[35:50] = True
    return A, tmask, omask


def test_gradient_matches_finite_differences():
    A, tm, om = _problem()
    rng = np.random.default_rng(3)
    x = rng.uniform(5, 50, A[0].shape[0])
    args = (tm, om, 1.0, 1.0, 0.4, 5.0)
    F, g = O.objective_grad(A, x, *args)
    h = 1e-4
    for j in range(len(x)):
        e = np.zeros_like(x)
        e[j] = h
        fd = (O.objective_grad(A, x + e, *args)[0] - O.objective_grad(A, x - e, *args)[0]) / (2 * h)
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_lipschitz_bound_is_the_largest_eigenvalue():
    A, tm, om = _problem()
    m = tm * 1.0 + om * 5.0
    H = sum(As.toarray() @ np.diag(m) @ As.toarray().T for As in A) * 2.0 / len(A)
    lam = np.linalg.eigvalsh(H).max()
    L = O.lipschitz(A, tm, om, 1.0, 5.0, n_power=200)
    assert L == pytest.approx(1.05 * lam, rel=1e-6)


def test_fista_reaches_the_nnls_optimum():
    A, _, _ = _problem(seed=1, S=2)
    nvox = A[0].shape[1]
    tm = np.ones(nvox, bool)
    om = np.zeros(nvox, bool)
    dp = 1.0
    # stacked least squares: min_x sum_s ||A_s^T x - dp||^2, x >= 0
    M = np.vstack([As.toarray().T for As in A])
    b = np.full(M.shape[0], dp)
    x_star, _ = nnls(M, b)
    F_star = np.sum((M @ x_star - b) ** 2) / len(A)
    x, hist, L = O.fista(A, np.ones(A[0].shape[0]), tm, om, dp, 1.0, 0.0, 0.0, iters=3000)
    assert hist[-1] == pytest.approx(O.objective_grad(A, x, tm, om, dp, 1.0, 0.0, 0.0)[0], rel=1e-15)
    F_end = O.objective_grad(A, x, tm, om, dp, 1.0, 0.0, 0.0)[0]
    assert F_end == pytest.approx(F_star, rel=1e-6)
    assert np.allclose(x, x_star, rtol=1e-3, atol=1e-3 * x_star.max())


def test_no_curvature_leaves_the_projected_start():
    """Empty structures: the eigenvalue is 0 and every step only projects."""
    A, _, _ = _problem(seed=2)
    n = A[0].shape[0]
    z = np.zeros(A[0].shape[1], bool)
    x0 = np.linspace(-1.0, 1.0, n)
    x, hist, L = O.fista(A, x0, z, z, 1.0, 1.0, 0.5, 1.0, iters=5)
    assert L == 0.0
    assert np.array_equal(x, np.maximum(x0, 0.0))
    assert np.all(hist == 0.0)


def test_matrices_from_csr_layout():
    """A field's rows inside the (scenario, field, spot) layout."""
    from paper_2307_01416_amd import inputs as I
    P = I.opt_problem(seed=4, n_spots=10, n_scen=2)
    # the 10 spots as two fields of 4 and 6: field 1 = offset 4, stride 10
    A = O.matrices_from_csr(P.row_ptr, P.col, P.val, 2, 6, P.nvox, row_stride=10, row_offset=4)
    full = O.matrices_from_csr(P.row_ptr, P.col, P.val, 2, 10, P.nvox)
    for s in range(2):
        assert (A[s] != full[s][4:]).nnz == 0
