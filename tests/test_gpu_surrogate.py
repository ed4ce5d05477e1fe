"""GPU checks of the surrogate network kernels (BF16 matrix cores, FP32
accumulation) against the FP64 oracle network: forward outputs and loss
gradients agree to BF16 precision (relative L2 <= 2e-2, cosine > 0.999), the
GPU's Adam update matches the oracle's element by element, and training on
the GPU lowers the loss."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2307_01416_amd import vpmc as V
    c = V.vpmc_create(0)
    yield c
    V.vpmc_destroy(c)


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 8))
    t = (rng.uniform(size=n) < 0.5).astype(np.float64)
    y = np.stack([0.3 * x[:, 0] + 0.1 * rng.normal(size=n), 0.5 * np.abs(x[:, 1]) + 0.1 * rng.normal(size=n),
                  0.2 * x[:, 2] ** 2 + 0.1 * rng.normal(size=n)], 1)
    return x, y, t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_forward_matches_oracle(ctx, orc):
    from paper_2307_01416_amd import vpmc as V
    assert V.vpmc_surrogate_param_count() == orc.mlp_num_params()
    p = orc.mlp_init(3)
    V.vpmc_surrogate_set_weights(ctx, p)
    assert np.array_equal(V.vpmc_surrogate_get_weights(ctx), p.astype(np.float32))
    x, _, _ = _data(300)          # not a multiple of the 64-row tile
    out = V.vpmc_surrogate_forward(ctx, x)
    ref = orc.mlp_forward(p, x)
    say(f"  forward rel L2 {_rel(out, ref):.3e} cosine {_cos(out.ravel(), ref.ravel()):.6f}")
    assert _rel(out, ref) <= 2e-2 and _cos(out.ravel(), ref.ravel()) > 0.999


@pytest.mark.parametrize("n", [1000, 4096])   # ragged tiles and K split; the training batch
def test_gradient_matches_oracle(ctx, orc, n):
    from paper_2307_01416_amd import vpmc as V
    p = orc.mlp_init(5) * 0.5
    V.vpmc_surrogate_set_weights(ctx, p)
    x, y, t = _data(n, seed=1)
    lg, gg = V.vpmc_surrogate_loss_grad(ctx, x, y, t)
    lo, go = orc.mlp_loss_grad(p, x, y, t)
    say(f"  loss gpu {lg:.6f} oracle {lo:.6f}; grad rel L2 {_rel(gg, go):.3e} cosine {_cos(gg, go):.6f}")
    assert lg == pytest.approx(lo, rel=1e-2)
    assert _rel(gg, go) <= 2e-2 and _cos(gg, go) > 0.999
    # per layer too (the input layer sees the most rounding)
    off = 0
    for ni, no in zip(orc.MLP_DIMS[:-1], orc.MLP_DIMS[1:]):
        sl = slice(off, off + no * ni + no)
        assert _cos(gg[sl], go[sl]) > 0.995, (ni, no)
        off += no * ni + no


def test_training_lowers_loss(ctx, orc):
    from paper_2307_01416_amd import vpmc as V
    V.vpmc_surrogate_set_weights(ctx, orc.mlp_init(7) * 0.5)
    x, y, t = _data(16384, seed=2)
    losses = V.vpmc_surrogate_train(ctx, x, y, t, epochs=8, batch=1024, lr=1e-3, seed=0)
    say(f"  training losses {np.round(losses, 4)}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0]
    # the trained weights agree with a forward pass of the oracle
    w = V.vpmc_surrogate_get_weights(ctx)
    out = V.vpmc_surrogate_forward(ctx, x[:256])
    ref = orc.mlp_forward(w.astype(np.float64), x[:256])
    assert _rel(out, ref) <= 3e-2


def test_adam_steps_match_oracle(ctx, orc):
    """The GPU's FP32 Adam update against the oracle's FP64 mlp_adam_step
    (Kingma & Ba, bias-corrected moments) applied to the GPU's own gradient,
    element by element, for the first two steps (one full batch per epoch,
    so each epoch is one step; the moments carry over)."""
    import ctypes as C
    from paper_2307_01416_amd import vpmc as V

    def P(a):
        return a.ctypes.data_as(C.c_void_p)

    w = (orc.mlp_init(11) * 0.5).astype(np.float32)
    V.vpmc_surrogate_set_weights(ctx, w)        # moments cleared, step count 0
    x, y, t = _data(1024, seed=4)
    lr = 1e-3
    n = w.size
    m, v = np.zeros(n), np.zeros(n)
    prev = w.astype(np.float64)
    for step in (1, 2):
        _, g = V.vpmc_surrogate_loss_grad(ctx, x, y, t)        # at the GPU's current weights
        V.vpmc_surrogate_train(ctx, x, y, t, epochs=1, batch=1024, lr=lr, seed=step)
        got = V.vpmc_surrogate_get_weights(ctx).astype(np.float64)
        ref = prev.copy()
        gd = np.ascontiguousarray(g, dtype=np.float64)
        orc.lib().mlp_adam_step(P(ref), P(gd), P(m), P(v), n, step, lr, 0.9, 0.999, 1e-8)
        d_got, d_ref = got - prev, ref - prev
        # the training pass sums the batch in another sample order than
        # loss_grad: elements whose gradient is not far above that rounding
        # may move differently; every other element moves as the oracle says
        big = np.abs(gd) > 1e-5
        err = np.abs(d_got - d_ref)[big]
        say(f"  Adam step {step}: {int(big.sum())} of {n} elements, max |dw - dw_ref| {err.max():.3e} "
            f"(lr {lr}), rel L2 of the whole update {_rel(d_got, d_ref):.2e}")
        assert np.all(err <= 1e-3 * lr + 2.0 ** -22 * np.abs(got[big]))
        assert _rel(d_got, d_ref) <= 1e-3
        prev = got


def _oracle_targets(ent, out, thick=30.0):
    """Targets of the network computed from the oracle's traversals."""
    e0 = ent[:, 4]
    u0, v0 = ent[:, 2], ent[:, 3]
    w0 = np.sqrt(1 - u0 ** 2 - v0 ** 2)
    frac = (e0 - out[:, 1]) / e0
    cosang = np.clip(u0 * out[:, 2] + v0 * out[:, 3] + w0 * out[:, 4], -1, 1)
    xs = ent[:, 0] + thick * u0 / w0
    ys = ent[:, 1] + thick * v0 / w0
    off = np.hypot(out[:, 5] - xs, out[:, 6] - ys)
    return np.stack([(frac - 0.5) / 0.25, np.arccos(cosang) / 0.05, off / 2.0], 1)


def test_training_data_matches_oracle_traversals(orc):
    """The GPU sampler (plain brass transport, FP32) against the oracle's FP64
    traversals of the same entries: features agree, outcome fractions and
    target means per energy bin agree within 4 standard errors."""
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    c = I.config2(20.0, False, histories_per_case=1000)
    xy, ang, e = I.surrogate_training_entries(60000, seed=1, polygon=c.fields[0].polygon)
    ent = np.column_stack([xy, ang, e])
    eng = V.Engine(0)
    try:
        eng.load_case(c)
        x, y, t = V.vpmc_surrogate_sample(eng.ctx, 0, ent, seed=11)
    finally:
        eng.close()
    out = orc.block_traverse(c, ent, seed=12)
    # features: deterministic functions of the entry
    np.testing.assert_allclose(x[:, :5], np.column_stack([xy / 20, ang / 0.05, (e - 150) / 50]), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(x[:, 5], np.minimum(out[:, 7], 100) / 10, rtol=1e-4, atol=1e-4)
    near = out[:, 7] < 1e-3
    assert np.array_equal((t == -1)[~near], (out[:, 0] == -1)[~near])
    brass = out[:, 0] >= 0
    yo = _oracle_targets(ent, out)
    bins = np.linspace(71, 229, 9)
    for lo, hi in zip(bins[:-1], bins[1:]):
        m = brass & (e >= lo) & (e < hi)
        pg, po = np.mean(t[m] == 1), np.mean(out[m, 0] == 1)
        se = np.sqrt(max(po * (1 - po), 1e-4) * 2 / m.sum())
        say(f"  E [{lo:.0f},{hi:.0f}): transmitted gpu {pg:.4f} oracle {po:.4f}")
        assert abs(pg - po) <= 4 * se + 1e-3
        mg, mo = m & (t == 1), m & (out[:, 0] == 1)
        if mg.sum() > 200 and mo.sum() > 200:
            for j in range(3):
                a, b = y[mg, j], yo[mo, j]
                se = np.sqrt(a.var() / a.size + b.var() / b.size)
                assert abs(a.mean() - b.mean()) <= 4 * se + 1e-3, (lo, j, a.mean(), b.mean())


# ------------------------------------------------ surrogate inside the transport
def _q(eng, case, **kw):
    dose, sig, led = eng.run_dose(case, **kw)
    q, k = eng.last_tally(0)
    from paper_2307_01416_amd import vpmc as V
    return q.cpu().numpy(), k, dose[0].cpu().numpy(), (None if sig is None else sig[0].cpu().numpy()), led[0], \
        V.vpmc_last_stats(eng.ctx)


def test_surrogate_is_a_noop_without_block():
    """No aperture: no VP is deferred and the tally is bitwise the plain one."""
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    c = I.config1(n_histories=50_000)
    eng = V.Engine(0)
    try:
        eng.load_case(c)
        V.vpmc_surrogate_set_weights(eng.ctx, V.surrogate_init(1))
        say("case config1 surrogate no-op")
        qa, ka, _, _, la, _ = _q(eng, c, n_batches=0, sigma=False)
        qb, kb, _, _, lb, st = _q(eng, c, n_batches=0, sigma=False, surrogate=True)
    finally:
        eng.close()
    assert st["deferred"] == 0
    assert ka == kb and np.array_equal(qa, qb) and np.array_equal(la, lb)


def test_surrogate_uncertain_band_resumes_plain_bitwise():
    """With the whole probability range marked uncertain every deferred VP is
    resumed by the plain brass transport from its recorded state: the tally
    equals the run without the surrogate bit for bit."""
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    c = I.config2(10.0, True, histories_per_case=200_000, shape=(64, 64, 200))
    eng = V.Engine(0)
    try:
        eng.load_case(c)
        V.vpmc_surrogate_set_weights(eng.ctx, V.surrogate_init(2))
        V.vpmc_surrogate_config(eng.ctx, 0.0, 0.0, 1.0)
        say("case config2 10mm RS surrogate identity band")
        qa, ka, _, _, la, sa = _q(eng, c, n_batches=4, sigma=False)
        qb, kb, _, _, lb, sb = _q(eng, c, n_batches=4, sigma=False, surrogate=True)
    finally:
        eng.close()
    say(f"  deferred {sb['deferred']} of {sb['histories']} VPs")
    assert sb["deferred"] > 0.2 * sb["histories"]
    assert sa["steps"] == sb["steps"] and sa["histories"] == sb["histories"]
    assert ka == kb and np.array_equal(qa, qb) and np.array_equal(la, lb)


@pytest.mark.parametrize("opening,rs,energy", [(10.0, True, None), (20.0, False, 215.0)])
def test_trained_surrogate_matches_plain_transport(opening, rs, energy):
    """Surrogate trained on the GPU (plain-transport traversals, BF16 matrix
    cores) against the plain transport, independent seeds: >= 99 % of voxels
    above 10 % of the maximum within 3 combined standard errors, gamma
    1 %/1 mm >= 99 %, high-dose mean within 0.5 % (or 3 s.e.).  Reports the
    share of VPs the network took and the transport time of both runs."""
    from gamma import gamma_pass_rate
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    c = I.config2(opening, rs, histories_per_case=10_000_000, shape=(64, 64, 200))
    if energy is not None:
        c.fields[0].spots["energy_mev"] = energy
        c.fields[0].spots["sigma_mm"] = I.spot_sigma_mm(energy)
    eng = V.Engine(0)
    try:
        say(f"case surrogate training for opening={opening} rs={rs} energy={energy}")
        losses = eng.train_surrogate(c, n=2_000_000, epochs=6, seed=3)
        say(f"  training losses {np.round(losses, 4)}")
        assert np.all(np.isfinite(losses)) and losses[-1] < losses[0]
        V.vpmc_surrogate_config(eng.ctx)
        _, _, dp, sp, lp, stp = _q(eng, c, n_batches=16, seed=0)
        _, _, ds, ss, ls, sts = _q(eng, c, n_batches=16, seed=1, surrogate=True)
    finally:
        eng.close()
    say(f"  plain {stp['transport_ms']:.1f} ms, surrogate {sts['transport_ms']:.1f} ms "
        f"({stp['transport_ms'] / sts['transport_ms']:.2f}x); deferred {sts['deferred']} of {sts['histories']} VPs; "
        f"steps {stp['steps']} -> {sts['steps']}")
    assert sts["deferred"] > 0
    m = dp >= 0.1 * dp.max()
    comb = np.sqrt(sp ** 2 + ss ** 2)
    frac = np.mean(np.abs(ds - dp)[m] <= 3.0 * comb[m])
    hi = dp >= 0.5 * dp.max()
    ratio = ds[hi].mean() / dp[hi].mean()
    se = np.sqrt(np.sum(sp[hi] ** 2 + ss[hi] ** 2)) / hi.sum() / dp[hi].mean()
    rate = gamma_pass_rate(dp, ds, c.geometry.spacing, 0.01, 1.0)
    say(f"  3-sigma fraction {frac:.4f}, mean-dose ratio {ratio:.5f} (s.e. {se:.4f}), gamma 1%/1mm {rate:.4f}; "
        f"block ledger plain {lp[2]:.4g} surrogate {ls[2]:.4g} MeV")
    assert frac >= 0.99
    assert abs(ratio - 1.0) <= max(0.005, 3.0 * se)
    assert rate >= 0.99


def test_surrogate_uncertain_band_csr_bitwise():
    """Influence-matrix (work-queue) runs: with the whole probability range
    uncertain, deferral and resume into the rows' sparse slots give the same
    rows, values and ledgers as the run without the surrogate."""
    from paper_2307_01416_amd import inputs as I
    from paper_2307_01416_amd import vpmc as V
    c = I.config2(10.0, True, histories_per_case=100_000, shape=(64, 64, 200))
    c.scenarios = [I.Scenario(), I.Scenario(shift_mm=(3.0, 0.0, 0.0), range_scale=1.035)]
    eng = V.Engine(0)
    try:
        eng.load_case(c)
        V.vpmc_surrogate_set_weights(eng.ctx, V.surrogate_init(4))
        V.vpmc_surrogate_config(eng.ctx, 0.0, 0.0, 1.0)
        say("case config2 10mm RS CSR surrogate identity band")
        rp0, col0, _, q0, k0 = eng.run_csr(c)
        l0 = eng.last_ledger.copy()
        rp1, col1, _, q1, k1 = eng.run_csr(c, surrogate=True)
        st = V.vpmc_last_stats(eng.ctx)
        l1 = eng.last_ledger.copy()
    finally:
        eng.close()
    say(f"  deferred {st['deferred']} of {st['histories']} VPs, nnz {rp1[-1]}")
    assert st["deferred"] > 0.2 * st["histories"]
    assert k0 == k1
    assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1) and np.array_equal(q0, q1)
    assert np.array_equal(l0, l1)


def test_fused_inference_throughput_and_agreement(orc):
    """The fused inference kernel on a large batch: outputs agree with the
    FP64 reference network to BF16 precision on a sample, and it runs at a
    reported fraction of the BF16 matrix-core peak."""
    import time
    import torch
    from paper_2307_01416_amd import vpmc as V
    c = V.vpmc_create(0)
    try:
        p = orc.mlp_init(9)
        V.vpmc_surrogate_set_weights(c, p)
        rng = np.random.default_rng(4)
        n = 1 << 20
        x = rng.normal(size=(n, 8)).astype(np.float32)
        V.vpmc_surrogate_forward(c, x[:4096])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = V.vpmc_surrogate_forward(c, x)
        dt = time.perf_counter() - t0
    finally:
        V.vpmc_destroy(c)
    flops = 2.0 * n * (8 * 256 + 3 * 256 * 256 + 256 * 29)
    say(f"  fused inference of {n} samples: {dt * 1e3:.1f} ms incl. host copies, {flops / dt / 1e12:.1f} TFLOP/s")
    idx = rng.choice(n, 512, replace=False)
    ref = orc.mlp_forward(p, x[idx].astype(np.float64))
    assert _rel(out[idx], ref) <= 2e-2 and _cos(out[idx].ravel(), ref.ravel()) > 0.999
    assert np.all(np.isfinite(out))
