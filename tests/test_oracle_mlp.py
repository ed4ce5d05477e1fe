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


def test_forward_layout_one_hot_path(orc):
    """Weights W[out][in] then b[out], layer by layer: a single non-zero
    weight per layer routes input 3 through four SiLU units to output 7, so
    out[7] = silu^4(x3) (silu(z) = z * logistic(z)), out[j] = b_j elsewhere."""
    from scipy.special import expit
    dims = orc.MLP_DIMS
    p = np.zeros(orc.mlp_num_params())
    off = 0
    picks = [(5, 3), (9, 5), (2, 9), (200, 2), (7, 200)]   # (out, in) per layer
    for (ni, no), (o, i) in zip(zip(dims[:-1], dims[1:]), picks):
        p[off + o * ni + i] = 1.0
        off += no * ni + no
    p[-29:] += np.linspace(-1.0, 1.0, 29) * (np.arange(29) != 7)
    x = np.zeros((2, 8))
    x[0, 3], x[1, 3] = 1.7, -0.6
    out = orc.mlp_forward(p, x)
    for r in range(2):
        z = x[r, 3]
        for _ in range(4):
            z = z * expit(z)
        assert out[r, 7] == pytest.approx(z, rel=1e-13)
        others = np.delete(out[r], 7)
        ref = np.delete(np.linspace(-1.0, 1.0, 29), 7)
        np.testing.assert_allclose(others, ref, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- Adam
# mlp_adam_step follows Kingma & Ba (ICLR 2015, Algorithm 1): biased moments
# m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, bias-corrected by
# 1 - b^t, step lr * m_hat / (sqrt(v_hat) + eps).  Closed forms pin it.
def _adam(orc, p, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
    import ctypes as C
    p = np.array(p, np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    for t, g in enumerate(grads, start=1):
        g = np.ascontiguousarray(g, np.float64)
        orc.lib().mlp_adam_step(P(p), P(g), P(m), P(v), p.size, t, lr, b1, b2, eps)
    return p


def test_adam_first_step_is_lr_times_sign(orc):
    # from zero moments the bias corrections make m_hat = g, v_hat = g^2
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=64)
    g = rng.normal(size=64) * 10.0 ** rng.uniform(-4, 1, size=64)
    p1 = _adam(orc, p0, [g], lr=1e-3)
    np.testing.assert_allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-18)


def test_adam_constant_gradient_steps_are_equal(orc):
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step t
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=32)
    g = rng.normal(size=32)
    p10 = _adam(orc, p0, [g] * 10, lr=2e-3)
    np.testing.assert_allclose(p10, p0 - 10 * 2e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-16)


def test_adam_alternating_gradient_momentum_closed_form(orc):
    # g_t = (-1)^t c: m_t = (1 - b1) c (-1)^t (1 - (-b1)^t) / (1 + b1),
    # v_t = c^2 (1 - b2^t), so v_hat = c^2 and the step is lr * m_hat_t / (c + eps)
    b1, b2, lr, c = 0.9, 0.999, 1e-2, 0.37
    T = 7
    p = _adam(orc, [0.0], [np.array([(-1) ** t * c]) for t in range(1, T + 1)], lr=lr, b1=b1, b2=b2)
    ref = 0.0
    for t in range(1, T + 1):
        m = (1 - b1) * c * (-1) ** t * (1 - (-b1) ** t) / (1 + b1)
        ref -= lr * (m / (1 - b1 ** t)) / (c + 1e-8)
    assert p[0] == pytest.approx(ref, rel=1e-13)
