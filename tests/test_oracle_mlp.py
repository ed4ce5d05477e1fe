"""Pins of the surrogate network's FP64 reference: the gradient equals central
finite differences of the loss, and the loss of a one-component mixture is
the Gaussian negative log likelihood computed by scipy."""
import numpy as np
import pytest
from scipy import stats


def _batch(rng, n):
    x = rng.normal(size=(n, 8))
    y = rng.normal(size=(n, 3)) * 0.5
    t = (rng.uniform(size=n) < 0.6).astype(np.float64)
    return x, y, t


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    p = orc.mlp_init(1) * 0.5
    x, y, t = _batch(rng, 6)
    loss, g = orc.mlp_loss_grad(p, x, y, t)
    assert np.isfinite(loss)
    idx = rng.choice(p.size, 60, replace=False)
    # include the output layer's biases (transmission, weights, means, log-sigmas)
    idx = np.concatenate([idx, np.arange(p.size - 29, p.size)])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (orc.mlp_loss_grad(pp, x, y, t)[0] - orc.mlp_loss_grad(pm, x, y, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_single_component_loss_is_gaussian_nll(orc):
    # zero hidden weights: the outputs are the last layer's biases
    p = np.zeros(orc.mlp_num_params())
    b = p[-29:]
    b[0] = 0.3                     # transmission logit
    b[1:5] = [0.0, -50.0, -50.0, -50.0]
    b[5:8] = [0.1, -0.2, 0.3]      # mean of component 0
    b[17:20] = [-0.5, 0.0, 0.2]    # log sigma of component 0
    x = np.zeros((1, 8))
    y = np.array([[0.4, 0.1, -0.3]])
    loss, _ = orc.mlp_loss_grad(p, x, y, np.array([1.0]))
    bce = np.log1p(np.exp(-0.3))
    nll = -np.sum(stats.norm.logpdf(y[0], loc=b[5:8], scale=np.exp(b[17:20])))
    assert loss == pytest.approx(bce + nll, rel=1e-9)
    loss0, _ = orc.mlp_loss_grad(p, x, y, np.array([0.0]))
    assert loss0 == pytest.approx(0.3 + np.log1p(np.exp(-0.3)), rel=1e-12)
