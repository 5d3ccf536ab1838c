"""GPU parity of the learned splitter: forward pass and bucket ids bit-exact with the
FP32 reference, thresholds exact, gradients and an Adam step against the double
reference, the end-to-end learned sort bit-exact against the plain definition, and
the balance the trained model gains over the untrained one."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2205_05982_amd import workloads as W
from tests.helpers import to_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _params(seed, x0=0.53, xs=6.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.NBLOCK)
    p[mlp.SL["w1"]] = rng.uniform(1.0, 20.0, mlp.H)
    p[mlp.SL["b1"]] = rng.uniform(-10.0, 2.0, mlp.H)
    p[mlp.SL["W2"]] = rng.uniform(0.0, 0.12, mlp.H * mlp.H)
    p[mlp.SL["b2"]] = rng.uniform(-0.5, 0.3, mlp.H)
    p[mlp.SL["w3"]] = rng.uniform(0.0, 0.08, mlp.H)
    p[mlp.SL["b3"]] = 0.05
    p[mlp.X0], p[mlp.XS] = x0, xs
    return p.astype(np.float32)


def test_forward_bit_exact(vqs):
    import torch
    p = _params(1)
    x = np.random.default_rng(2).uniform(0.5, 0.8, 100_000).astype(np.float32)
    y = to_host(vqs.mlp_forward(to_gpu(p), to_gpu(x)))
    np.testing.assert_array_equal(y, mlp.forward_f32(p, x))


def test_buckets_bit_exact_and_thresholds_exact(vqs):
    import torch
    for seed in (3, 4):
        p = _params(seed)
        keys = W.lognormal_mixture_u64(300_000, 15)
        keys = np.concatenate([keys, np.array([0, 1, 2**64 - 1], dtype=np.uint64)])
        kg = to_gpu(keys)
        pg = to_gpu(p)
        b_gpu = to_host(vqs.mlp_buckets(pg, kg))
        np.testing.assert_array_equal(b_gpu, mlp.buckets_f32(p, keys))
        thr, nv = vqs.learned_thresholds(pg)
        b_thr = to_host(vqs.learned_classify(kg, thr, nv))
        np.testing.assert_array_equal(b_thr, b_gpu)
        # thresholds are the first keys of their buckets
        t = to_host(thr).view(np.uint64)[: int(to_host(nv)[0])]
        assert (np.diff(t.astype(object)) >= 0).all()
        j = np.arange(1, t.size + 1)
        assert (mlp.buckets_f32(p, t) >= j).all()            # t_j reaches bucket j ...
        prev = mlp.buckets_f32(p, t[t > 0] - np.uint64(1))
        assert (prev < j[t > 0]).all()                      # ... and t_j - 1 does not


def test_gradient_matches_double_reference(vqs):
    p = _params(5)
    rng = np.random.default_rng(6)
    x = rng.uniform(0.53, 0.69, 192).astype(np.float32)
    t = np.sort(rng.uniform(0, 1, 192)).astype(np.float32)
    g, loss = vqs.mlp_gradient(to_gpu(p), to_gpu(x), to_gpu(t))
    lw, gw = mlp.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    g = to_host(g).astype(np.float64)
    rel = np.linalg.norm(g - gw[:mlp.NPARAM]) / np.linalg.norm(gw[:mlp.NPARAM])
    assert rel < 1e-4, rel
    assert abs(float(to_host(loss)[0]) - lw) < 1e-6 + 1e-4 * lw


def test_one_adam_step_matches_reference(vqs):
    import torch
    p = _params(7)
    rng = np.random.default_rng(8)
    x = rng.uniform(0.53, 0.69, 192).astype(np.float32)
    t = np.sort(rng.uniform(0, 1, 192)).astype(np.float32)
    pg = to_gpu(p)
    mom = torch.zeros(2 * mlp.NPARAM + 1, dtype=torch.float32, device="cuda")
    vqs.mlp_train(pg, mom, to_gpu(x), to_gpu(t), steps=1, batch=192, lr=1e-3, sequential=True)
    _, g = mlp.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    want, _, _ = mlp.adam_step(p.astype(np.float64), g, np.zeros(mlp.NBLOCK), np.zeros(mlp.NBLOCK), 1,
                               mlp.lr_at(1, 1, 1e-3))
    got = to_host(pg).astype(np.float64)
    # the first Adam step moves each parameter by ~lr * sign(g): compare where |g| is
    # clearly nonzero (where it is tiny, FP32 rounding can flip the step)
    sel = np.abs(g[:mlp.NPARAM]) > 1e-5
    np.testing.assert_allclose(got[:mlp.NPARAM][sel], want[:mlp.NPARAM][sel], rtol=1e-5, atol=1e-6)


def test_init_matches_reference(vqs):
    import torch
    x = np.sort(np.random.default_rng(9).uniform(0.55, 0.7, 1000)).astype(np.float32)
    pg = torch.empty(mlp.NBLOCK, dtype=torch.float32, device="cuda")
    vqs.mlp_init(pg, 16, to_gpu(x))
    x0 = np.float32(x[0])
    xs = np.float32(1.0) / (np.float32(x[-1]) - x0)
    np.testing.assert_array_equal(to_host(pg), mlp.init_params(16, x0, xs).astype(np.float32))


@pytest.mark.parametrize("n", [2_000_000, 5_000_000])
def test_learned_sort_bit_exact(vqs, n):
    import torch
    keys = W.lognormal_mixture_u64(n, 15)
    t = to_gpu(keys)
    vqs.sort(t, key_type=3, method=1)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), np.sort(keys))
    st = vqs.get_stats()
    assert st["learned_buckets"] == 256 and st["max_bucket"] > 0


def test_learned_sort_overflow_rule_and_degenerate_inputs(vqs):
    import torch
    for keys in (W.few_distinct_u64(1_000_000, 4), np.full(200_000, 5, dtype=np.uint64),
                 W.uniform_u64(1_000_000, 2)):
        t = to_gpu(keys)
        vqs.sort(t, key_type=3, method=1, overflow_factor=0.5)
        torch.cuda.synchronize()
        assert vqs.last_error_bits() == 0
        np.testing.assert_array_equal(to_host(t), np.sort(keys))
        st = vqs.get_stats()
        assert st["overflow_buckets"] >= 1


def test_trained_model_balances_better_than_untrained(vqs):
    """Bucket balance on the mixture workload (4e6 keys) of (A) the model trained with
    the default settings, (B) the untrained model, and, as the yardstick, (C) the 256
    ranges that 8 levels of the paper's plain pivot sampling make."""
    import torch
    n = 4_000_000
    keys = W.lognormal_mixture_u64(n, 15)
    kg = to_gpu(keys)
    trained = vqs.learned_fit(kg)
    p = to_host(trained)
    untrained = mlp.init_params(16, np.float32(p[mlp.X0]), np.float32(p[mlp.XS])).astype(np.float32)
    bt = np.bincount(to_host(vqs.mlp_buckets(trained, kg)), minlength=256)
    bu = np.bincount(to_host(vqs.mlp_buckets(to_gpu(untrained), kg)), minlength=256)
    plain = oracle.plain_split_sizes(keys, W.U64, levels=8)
    jt, ju = mlp.balance(bt, n), mlp.balance(bu, n)
    jp = {"max_over_expected": float(plain.max() / (n / 256)), "ranges": int(plain.size)}
    print("trained", jt, "untrained", ju, "plain 8 levels", jp)
    assert jt["rms_rel_dev"] < 0.75 * ju["rms_rel_dev"]
    assert bt.max() < bu.max()
    # no bucket of the trained model beyond what plain sampling's worst range holds
    assert bt.max() <= plain.max()


def test_fit_sample_targets_and_first_step_match_reference(vqs):
    """learned_fit with one Adam step against the same steps on the CPU: the sampled
    64-byte chunks (SplitMix64 outputs of the sample seed), their sort, x(k) and the
    mid-rank targets (runs of equal keys included: the mixture has Zipf duplicates),
    the untrained model, the minibatch draw and the step."""
    n, seed_s, seed_m, batch, lr = 3_000_000, 17, 16, 256, 0.003
    keys = W.lognormal_mixture_u64(n, 15)
    params = to_host(vqs.learned_fit(to_gpu(keys), train_steps=1, batch=batch))
    # sample: chunks = floor(frac * n / 8) with the FP32 default fraction 0.01
    chunks = int(float(np.float32(0.01)) * n / 8.0)
    chunks = min(max(chunks, 8), n // 8)
    m, nch = chunks * 8, n // 8
    u = np.array(oracle.splitmix64(seed_s, chunks), dtype=np.uint64) >> np.uint64(32)
    off = np.array([(int(v) * nch) >> 32 for v in u], dtype=np.int64) * 8
    s = np.sort(keys[off[:, None] + np.arange(8)].ravel())
    x = mlp.key_to_x(s).astype(np.float32)
    t = mlp.mid_rank_targets(s).astype(np.float32)
    assert np.unique(s).size < m                      # equal keys occur in the sample
    x0 = np.float32(x[0])
    xs = np.float32(1.0) / (np.float32(x[-1]) - x0)
    p0 = mlp.init_params(seed_m, x0, xs).astype(np.float32)
    np.testing.assert_array_equal(params[mlp.X0:], p0[mlp.X0:])
    draws = np.array(oracle.splitmix64(seed_s, batch), dtype=np.uint64) >> np.uint64(32)
    idx = np.array([(int(d) * m) >> 32 for d in draws])
    _, g = mlp.loss_and_grad(p0.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64))
    want, _, _ = mlp.adam_step(p0.astype(np.float64), g, np.zeros(mlp.NBLOCK), np.zeros(mlp.NBLOCK), 1,
                               mlp.lr_at(1, 1, lr))
    sel = np.abs(g[:mlp.NPARAM]) > 1e-5
    assert sel.sum() > 100
    np.testing.assert_allclose(params[:mlp.NPARAM][sel].astype(np.float64), want[:mlp.NPARAM][sel],
                               rtol=1e-5, atol=1e-6)
