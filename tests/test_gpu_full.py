"""Full-size parity: every workload at its full size (1e8 to 6.1e9 keys), sorted in the
default launch configuration that bench.py times.

The oracle cannot sort these sizes within a test, so the checks are
  * on the GPU, properties that hold at any size: the output is non-decreasing in the
    key order (within every segment for the batch) and holds the input's multiset (sum
    and sum of squares of the keys' bit patterns, mod 2^64, per word);
  * on the host, sampled outputs checked one by one against the input: out[r] is the
    r-th smallest key exactly when #{k < out[r]} <= r < #{k <= out[r]};
  * for the batch of 65,536 segments, whole sampled segments (the longest, the
    shortest and 20 random ones) against the oracle, element by element;
  * for the learned splitter, the output is identical to the plain method's.
"""
import numpy as np
import pytest

import oracle
from paper_2205_05982_amd import workloads as W
from tests.helpers import F32, F64, U16, U32, U64, U128, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _words(t, kt):
    """int64 words of the keys' bit patterns (one column, two for u128)."""
    import torch
    if kt == U128:
        tv = t.view(torch.int64)
        return [tv[:, 0], tv[:, 1]]
    if kt in (U64, F64):
        return [t.view(torch.int64)]
    if kt in (U32, F32):
        return [t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF]
    return [t.view(torch.int16).to(torch.int64) & 0xFFFF]


def _order_key(t, kt):
    """Tensors comparing like the keys (most significant first)."""
    import torch
    sign = torch.tensor(-(2**63), dtype=torch.int64, device=t.device)
    if kt in (F32, F64):
        return [t]
    if kt == U128:
        tv = t.view(torch.int64)
        return [tv[:, 1] ^ sign, tv[:, 0] ^ sign]
    if kt == U64:
        return [t.view(torch.int64) ^ sign]
    return _words(t, kt)


def _nondecreasing(t, kt):
    """Positions i with out[i] > out[i + 1]: a boolean tensor of length n - 1."""
    ks = _order_key(t, kt)
    if len(ks) == 1:
        return ks[0][1:] < ks[0][:-1]
    hi, lo = ks
    return (hi[1:] < hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] < lo[:-1]))


def _multiset_equal(a, b, kt):
    ok = True
    for x, y in zip(_words(a, kt), _words(b, kt)):
        ok &= bool((x.sum() == y.sum()).item()) and bool(((x * x).sum() == (y * y).sum()).item())
    return ok


def _host_less(host, v, kt, equal_too):
    if kt == U128:
        hi, lo = host[:, 1], host[:, 0]
        vlo, vhi = v[0], v[1]
        lt = (hi < vhi) | ((hi == vhi) & (lo < vlo))
        if equal_too:
            lt |= (hi == vhi) & (lo == vlo)
        return int(np.count_nonzero(lt))
    return int(np.count_nonzero(host <= v if equal_too else host < v))


def _check_sampled_ranks(host, out, kt, nranks=8, seed=0):
    n = host.shape[0]
    rng = np.random.default_rng(seed)
    ranks = sorted(set([0, n - 1, n // 2] + list(rng.integers(0, n, nranks))))
    for r in ranks:
        v = out[r].cpu().numpy()
        below, upto = _host_less(host, v, kt, False), _host_less(host, v, kt, True)
        assert below <= r < upto, (r, v, below, upto)


def _full_check(vqs, host, kt, **opts):
    import torch
    src = to_gpu(host)
    t = src.clone()
    vqs.sort(t, key_type=kt, **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    assert int(_nondecreasing(t, kt).sum().item()) == 0
    assert _multiset_equal(t, src, kt)
    _check_sampled_ranks(host, t, kt)
    return t, src


@pytest.mark.parametrize("dist", W.C2_DISTRIBUTIONS)
def test_c2_full_1e8_u64(vqs, dist):
    print(f"case: C2 {dist} 1e8 u64", flush=True)
    host = W.c2(dist, 100_000_000)
    _full_check(vqs, host, U64)
    st = vqs.get_stats()
    assert st["fallbacks"] == 0 or dist in ("zipf",)


@pytest.mark.parametrize("name", list(W.C3_CASES))
def test_c3_full_key_types(vqs, name):
    kt, gen, n = W.C3_CASES[name]
    print(f"case: C3 {name} {n:.1e}", flush=True)
    _full_check(vqs, gen(n), kt)


@pytest.mark.parametrize("kt", [U32, U64])
def test_c4_full_batch_65536_segments(vqs, kt):
    import torch
    off = W.segment_offsets(65536, 12)
    n = int(off[-1])
    bits, seed = (32, 13) if kt == U32 else (64, 14)
    print(f"case: C4 65536 segments, {n} keys, kt {kt}", flush=True)
    src = W.counter_torch(seed, 0, n, bits, "cuda")
    t = src.clone()
    o = to_gpu(off)
    vqs.sort_segmented(t, o, key_type=kt, use_graph=1)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    vt = W.U32 if kt == U32 else W.U64
    bad = _nondecreasing(t, vt)
    bad[o[1:-1] - 1] = False                 # pairs across a segment boundary
    assert int(bad.sum().item()) == 0
    del bad
    assert _multiset_equal(t, src, vt)
    del src
    lens = np.diff(off)
    rng = np.random.default_rng(99)
    pick = sorted(set([int(np.argmax(lens)), int(np.argmin(lens))] + list(rng.integers(0, 65536, 20))))
    gen = W.counter_u32 if kt == U32 else W.counter_u64
    for i in pick:
        a, b = int(off[i]), int(off[i + 1])
        want = gen(seed, a, b - a)
        oracle.sort(want, kt)
        got = t[a:b].cpu().numpy().view(want.dtype)
        np.testing.assert_array_equal(got, want)


def test_c5_full_learned_equals_plain(vqs):
    import torch
    n = 500_000_000
    print("case: C5 5e8 mixture, learned and plain", flush=True)
    host = W.lognormal_mixture_u64(n, 15)
    learned, src = _full_check(vqs, host, U64, method=1)
    st = vqs.get_stats()
    assert st["learned_buckets"] == 256
    plain = src.clone()
    del src
    vqs.sort(plain, key_type=U64)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    assert torch.equal(plain, learned)
