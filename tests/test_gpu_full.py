"""Full-size parity: every workload at its full size (5e7 to 6.1e9 keys), sorted in the
default launch configuration that bench.py times, against the CPU oracle.

  * One array (the seven 1e8 u64 distributions, the five key-type workloads): the
    GPU output equals the oracle's sort of the same input element by element.  The
    oracle runs on the host's threads (oracle.parallel_sort: its top recursion levels
    as parallel tasks, then its sort of each remaining range); the sorted order is
    unique, so this is the oracle's result.  For the benchmarked workload (1e8 u64
    uniform) the one-threaded oracle also gives the eight recursion counters, which
    equal the GPU's (same pivots at every level of the default configuration: 32K
    solo threshold, run-mode levels).
  * The 65,536-segment batch (6.1e9 keys): properties that hold at any size on the
    GPU (each segment non-decreasing, the input's multiset by sums of the keys' bit
    patterns), and, element by element against the oracle, a contiguous block of
    segments holding about 1e8 keys plus the longest, the shortest and 20 random
    segments (keys are SplitMix64 outputs by index, regenerated on the host).
  * The learned splitter at 5e8 keys: the output equals the oracle's sort; the bucket
    counts of the GPU's trained model, found by the oracle's FP32 forward pass on the
    oracle-sorted keys (bisection, exact because the bucket map is non-decreasing),
    give the largest bucket and the overflow count the GPU reports.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2205_05982_amd import workloads as W
from tests.helpers import F32, F64, U16, U32, U64, U128, assert_stats_equal, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _threads() -> int:
    t = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        t = min(t, int(cap))
    return max(t, 1)


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


def _nondecreasing_violations(t, kt):
    """Positions i with out[i] after out[i + 1]: a boolean tensor of length n - 1."""
    import torch
    sign = torch.tensor(-(2**63), dtype=torch.int64, device=t.device)
    if kt in (F32, F64):
        return t[1:] < t[:-1]
    if kt == U128:
        tv = t.view(torch.int64)
        hi, lo = tv[:, 1] ^ sign, tv[:, 0] ^ sign
        return (hi[1:] < hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] < lo[:-1]))
    k = t.view(torch.int64) ^ sign if kt == U64 else _words(t, kt)[0]
    return k[1:] < k[:-1]


def _multiset_equal(a, b, kt):
    ok = True
    for x, y in zip(_words(a, kt), _words(b, kt)):
        ok &= bool((x.sum() == y.sum()).item()) and bool(((x * x).sum() == (y * y).sum()).item())
    return ok


def _gpu_sort(vqs, host, kt, **opts):
    import torch
    t = to_gpu(host)
    vqs.sort(t, key_type=kt, **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    st = vqs.get_stats()
    out = t.cpu().numpy()
    del t
    torch.cuda.empty_cache()
    return out, st


def _oracle_sorted(host, kt):
    want = host.copy()
    oracle.parallel_sort(want, kt, _threads())
    return want


@pytest.mark.parametrize("dist", W.C2_DISTRIBUTIONS)
def test_c2_full_1e8_u64(vqs, dist):
    print(f"case: C2 {dist} 1e8 u64", flush=True)
    host = W.c2(dist, 100_000_000)
    got, st = _gpu_sort(vqs, host, U64)
    if dist == "uniform":
        # the benchmarked workload: the one-threaded oracle, with its recursion counters
        want = host.copy()
        ost = oracle.sort(want, U64, stats=True)
        assert_stats_equal(ost, st)
        assert st["levels"] >= 10      # the default configuration takes device-wide levels
    else:
        want = _oracle_sorted(host, U64)
    np.testing.assert_array_equal(got, want)
    assert st["fallbacks"] == 0 or dist in ("zipf",)


@pytest.mark.parametrize("name", list(W.C3_CASES))
def test_c3_full_key_types(vqs, name):
    kt, gen, n = W.C3_CASES[name]
    print(f"case: C3 {name} {n:.1e}", flush=True)
    host = gen(n)
    got, st = _gpu_sort(vqs, host, kt)
    np.testing.assert_array_equal(got, _oracle_sorted(host, kt))


def _oracle_segments(keys, off, kt):
    """The oracle's segmented sort, segments split over the host threads."""
    import concurrent.futures as cf
    nseg = off.size - 1
    parts = np.linspace(0, nseg, _threads() + 1).astype(np.int64)

    def run(i):
        a, b = int(parts[i]), int(parts[i + 1])
        if b > a:
            base = int(off[a])
            sub = keys[base:int(off[b])]
            oracle.sort_segmented(sub, off[a:b + 1] - base, kt)

    with cf.ThreadPoolExecutor(max_workers=_threads()) as ex:
        list(ex.map(run, range(parts.size - 1)))


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
    bad = _nondecreasing_violations(t, kt)
    bad[o[1:-1] - 1] = False                 # pairs across a segment boundary
    assert int(bad.sum().item()) == 0
    del bad
    assert _multiset_equal(t, src, kt)
    del src
    torch.cuda.empty_cache()
    gen = W.counter_u32 if kt == U32 else W.counter_u64
    # a contiguous block of segments holding about 1e8 keys, element by element
    s0 = 30_000
    s1 = int(np.searchsorted(off, off[s0] + 100_000_000))
    a, b = int(off[s0]), int(off[s1])
    want = gen(seed, a, b - a)
    _oracle_segments(want, off[s0:s1 + 1] - a, kt)
    got = t[a:b].cpu().numpy().view(want.dtype)
    np.testing.assert_array_equal(got, want)
    # the longest, the shortest and 20 random segments
    lens = np.diff(off)
    rng = np.random.default_rng(99)
    pick = sorted(set([int(np.argmax(lens)), int(np.argmin(lens))] + list(rng.integers(0, 65536, 20))))
    for i in pick:
        a, b = int(off[i]), int(off[i + 1])
        want = gen(seed, a, b - a)
        oracle.sort(want, kt)
        got = t[a:b].cpu().numpy().view(want.dtype)
        np.testing.assert_array_equal(got, want)


def _bucket_counts(params, sorted_keys):
    """Keys per bucket of the model, from the oracle's FP32 forward pass: the bucket map
    is non-decreasing in the key, so on sorted keys each bucket's first position is
    found by bisection."""
    n = sorted_keys.size
    bucket_at = lambda i: int(mlp.buckets_f32(params, sorted_keys[i:i + 1])[0])
    starts = np.zeros(257, dtype=np.int64)
    starts[256] = n
    for j in range(1, 256):
        lo, hi = 0, n                       # first position with bucket >= j
        while lo < hi:
            mid = (lo + hi) // 2
            if bucket_at(mid) >= j:
                hi = mid
            else:
                lo = mid + 1
        starts[j] = lo
    return np.diff(starts)


def test_c5_full_learned_against_the_oracle(vqs):
    import torch
    n = 500_000_000
    print("case: C5 5e8 mixture, learned", flush=True)
    host = W.lognormal_mixture_u64(n, 15)
    got, st = _gpu_sort(vqs, host, U64, method=1)
    assert st["learned_buckets"] == 256
    want = _oracle_sorted(host, U64)
    np.testing.assert_array_equal(got, want)
    del got
    # the bucket counts of the same trained model, by the oracle's forward pass
    t = to_gpu(host)
    params = vqs.learned_fit(t).cpu().numpy()
    del t
    torch.cuda.empty_cache()
    counts = _bucket_counts(params, want)
    assert counts.sum() == n
    assert st["max_bucket"] == int(counts.max())
    assert st["overflow_buckets"] == int(np.count_nonzero(counts.astype(np.float64) > 2.0 * n / 256))
    assert st["overflow_buckets"] >= 1        # the Zipf(1.2) duplicates overflow some bucket
