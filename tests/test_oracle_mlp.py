"""Pins of the learned-splitter reference (oracle/mlp.py, oracle/mlp_oracle.c).

Gradients against central finite differences, monotonicity of the bucket map,
closed forms of the targets and of Adam's first step, agreement of the FP32
fused-multiply-add forward with the double forward, and the exactness of
threshold compilation.
"""
import numpy as np
import pytest

from oracle import mlp


def _random_params(seed, x0=0.5, xs=4.0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.NBLOCK)
    p[mlp.SL["w1"]] = rng.uniform(1.0, 20.0, mlp.H) * scale
    p[mlp.SL["b1"]] = rng.uniform(-10.0, 2.0, mlp.H)
    p[mlp.SL["W2"]] = rng.uniform(0.0, 0.12, mlp.H * mlp.H)
    p[mlp.SL["b2"]] = rng.uniform(-0.5, 0.3, mlp.H)
    p[mlp.SL["w3"]] = rng.uniform(0.0, 0.08, mlp.H)
    p[mlp.SL["b3"]] = 0.05
    p[mlp.X0], p[mlp.XS] = x0, xs
    return p.astype(np.float32).astype(np.float64)


def test_gradient_matches_central_differences():
    p = _random_params(1)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.5, 0.75, 64)
    t = np.sort(rng.uniform(0, 1, 64))
    loss, g = mlp.loss_and_grad(p, x, t)
    h = 1e-6
    checked = 0
    for i in list(range(0, mlp.NPARAM, 7)) + [mlp.NPARAM - 1]:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = mlp.loss_and_grad(pp, x, t)
        lm, _ = mlp.loss_and_grad(pm, x, t)
        # skip parameters whose perturbation crosses a clamp kink
        _, cp = mlp.forward(pp, x)
        _, cm = mlp.forward(pm, x)
        kink = any(((np.asarray(a) > 0) & (np.asarray(a) < 1)).sum() != ((np.asarray(b) > 0) & (np.asarray(b) < 1)).sum()
                   for a, b in ((cp[1], cm[1]), (cp[3], cm[3]), (cp[5], cm[5])))
        if kink:
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])
        checked += 1
    assert checked > 100


def test_planted_sign_error_in_gradient_is_caught():
    p = _random_params(3)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.5, 0.75, 32)
    t = rng.uniform(0, 1, 32)
    _, g = mlp.loss_and_grad(p, x, t)
    i = mlp.SL["b3"].start
    h = 1e-6
    pp, pm = p.copy(), p.copy()
    pp[i] += h
    pm[i] -= h
    fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * h)
    assert abs(fd - g[i]) < 1e-6 and abs(fd + g[i]) > 1e-6     # a flipped sign would fail


def test_bucket_map_is_monotone_in_the_key():
    for seed in range(4):
        p = _random_params(seed, x0=0.53, xs=6.0)
        keys = np.sort(np.random.default_rng(seed).integers(0, 2**64, 200_000, dtype=np.uint64))
        keys = np.concatenate([np.arange(0, 5000, dtype=np.uint64), keys,
                               np.array([2**64 - 1], dtype=np.uint64)])
        b = mlp.buckets_f32(p, keys)
        assert (np.diff(b) >= 0).all()
        assert b.min() >= 0 and b.max() <= 255


def test_key_to_x_definition_and_monotonicity():
    k = np.array([0, 1, 2, 3, 2**24, 2**24 + 1, 2**63, 2**64 - 1], dtype=np.uint64)
    x = mlp.key_to_x(k)
    assert x[0] == 0.0
    # 1.0f has bits 0x3F800000
    assert x[1] == np.float32(0x3F800000) * np.float32(2.0 ** -31)
    assert x[4] == x[5]                       # 2^24 + 1 rounds to 2^24 in float32
    assert (np.diff(x.astype(np.float64)) >= 0).all()
    dense = np.sort(np.random.default_rng(0).integers(0, 2**64, 100_000, dtype=np.uint64))
    assert (np.diff(mlp.key_to_x(dense).astype(np.float64)) >= 0).all()


def test_fp32_forward_agrees_with_double_forward():
    p = _random_params(5, x0=0.55, xs=5.0)
    x = np.random.default_rng(6).uniform(0.5, 0.8, 10_000).astype(np.float32)
    y32 = mlp.forward_f32(p, x)
    y64, _ = mlp.forward(p, x.astype(np.float64))
    assert np.max(np.abs(y32 - y64)) < 2e-5


def test_thresholds_reproduce_the_bucket_map_exactly():
    p = _random_params(7, x0=0.53, xs=6.0)
    f = lambda k: int(mlp.buckets_f32(p, np.array([k], dtype=np.uint64))[0])
    J = f(2**64 - 1)
    thr = []
    for j in range(1, J + 1):
        lo, hi = 0, 2**64 - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if f(mid) >= j:
                hi = mid
            else:
                lo = mid + 1
        thr.append(lo)
    thr = np.array(thr, dtype=np.uint64)
    keys = np.random.default_rng(8).integers(0, 2**64, 50_000, dtype=np.uint64)
    keys = np.concatenate([keys, thr, thr - np.uint64(1), np.array([0, 2**64 - 1], dtype=np.uint64)])
    by_thr = np.searchsorted(thr, keys, side="right")
    np.testing.assert_array_equal(by_thr, mlp.buckets_f32(p, keys))


def test_mid_rank_targets_closed_forms():
    s = np.arange(10, dtype=np.uint64)
    np.testing.assert_allclose(mlp.mid_rank_targets(s), (np.arange(10) + 0.5) / 10)
    np.testing.assert_allclose(mlp.mid_rank_targets(np.full(7, 3, np.uint64)), 0.5)
    t = mlp.mid_rank_targets(np.array([1, 1, 2, 5, 5, 5], np.uint64))
    np.testing.assert_allclose(t, [1 / 6, 1 / 6, 2.5 / 6, 4.5 / 6, 4.5 / 6, 4.5 / 6])


def test_adam_first_step_closed_form_and_projection():
    p = _random_params(9)
    g = np.random.default_rng(10).standard_normal(mlp.NBLOCK) * 1e-2
    g[mlp.X0] = g[mlp.XS] = 0.0
    lr = 1e-3
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr)
    want = p - lr * mlp.lr_groups() * g / (np.abs(g) + 1e-8)
    for k in mlp.NONNEG:
        want[mlp.SL[k]] = np.maximum(want[mlp.SL[k]], 0.0)
    np.testing.assert_allclose(p1, want, rtol=0, atol=1e-12)
    assert (p1[mlp.SL["W2"]] >= 0).all()


def test_untrained_model_is_near_identity_on_xn():
    p = mlp.init_params(16, np.float32(0.5), np.float32(4.0))
    x = np.linspace(0.5, 0.75, 101)
    y, _ = mlp.forward(p, x)
    xn = (x - 0.5) * 4.0
    assert np.max(np.abs(y - xn)) < 0.06
    assert (p[mlp.SL["W2"]] > 0).all()


def test_learning_rate_schedule_endpoints_and_linearity():
    """The schedule's defining properties: lr at the first step, lr/10 at the last,
    equal decrements in between (a linear decay), and a lone step at lr."""
    lr, steps = 0.003, 100
    sched = np.array([mlp.lr_at(s, steps, lr) for s in range(1, steps + 1)])
    assert sched[0] == pytest.approx(lr, rel=1e-15)
    assert sched[-1] == pytest.approx(lr / 10, rel=1e-12)
    d = np.diff(sched)
    assert np.all(d < 0)
    np.testing.assert_allclose(d, d[0], rtol=1e-9)
    assert d.sum() == pytest.approx(-0.9 * lr, rel=1e-12)
    assert mlp.lr_at(1, 1, lr) == lr
