"""GPU parity: the HIP library against the CPU oracle, through the C interface.

Every case compares the sorted keys element by element (bit-exact: inputs hold no
NaN and no -0.0, so the sorted order is unique) and the recursion counters
(partitions, keys partitioned, degenerate partitions, all-equal ranges, base
cases, depth-limit fallbacks, maximum depth), which agree because the GPU uses
the oracle's pivot rule and partition layout at every level.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2205_05982_amd import workloads as W
from tests.helpers import (F32, F64, U16, U32, U64, U128, assert_stats_equal, random_keys, to_gpu,
                           to_host)

pytestmark = pytest.mark.gpu

TYPES = [U16, U32, U64, U128, F32, F64]


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _gpu_sort(vqs, keys, kt, asc=True, **opts):
    import torch
    t = to_gpu(keys)
    vqs.sort(t, ascending=asc, key_type=kt, **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    return to_host(t), vqs.get_stats()


def _check(vqs, keys, kt, asc=True, seed=0, depth_limit=-1, gpu_limit=0, **opts):
    want = keys.copy()
    ost = oracle.sort(want, kt, ascending=asc, seed=seed, depth_limit=depth_limit, stats=True)
    got, gst = _gpu_sort(vqs, keys, kt, asc, seed=seed, depth_limit=gpu_limit, **opts)
    np.testing.assert_array_equal(got, want)
    assert_stats_equal(ost, gst)
    return gst


def test_c1_one_million_u32_seed1(vqs):
    print("case: C1 1e6 u32", flush=True)
    _check(vqs, W.uniform_u32(1_000_000, 1), U32)


@pytest.mark.parametrize("kt", TYPES)
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("n", [1, 2, 17, 255, 256, 257, 1000, 2047, 2048, 4096, 4097, 8193,
                               16385, 50_000, 300_000])
def test_types_orders_sizes(vqs, kt, asc, n):
    print(f"case: kt={kt} asc={asc} n={n}", flush=True)
    _check(vqs, random_keys(kt, n, seed=1000 + n + kt), kt, asc, seed=n)


@pytest.mark.parametrize("kt", [U32, U64, F32])
def test_multi_level_sizes(vqs, kt):
    # large enough for several device-wide levels before the solo kernel
    n = 3_000_000
    print(f"case: multi-level kt={kt} n={n}", flush=True)
    gst = _check(vqs, random_keys(kt, n, seed=77), kt, seed=5, solo_max=20_000)
    assert gst["levels"] >= 3


@pytest.mark.parametrize("dist", W.C2_DISTRIBUTIONS)
def test_c2_distributions(vqs, dist):
    print(f"case: C2 {dist} 2e6", flush=True)
    _check(vqs, W.c2(dist, 2_000_000), U64, seed=3, solo_max=30_000)


@pytest.mark.parametrize("name", list(W.C3_CASES))
def test_c3_key_types(vqs, name):
    kt, gen, _ = W.C3_CASES[name]
    print(f"case: C3 {name} 1e6", flush=True)
    _check(vqs, gen(1_000_000), kt, seed=11)


def test_all_equal_and_two_values(vqs):
    _check(vqs, np.full(100_000, 7, dtype=np.uint64), U64)
    _check(vqs, np.full(100_000, 7, dtype=np.uint64), U64, asc=False)
    k = np.array([5] * 300_000 + [9] * 700_000, dtype=np.uint32)
    np.random.default_rng(0).shuffle(k)
    _check(vqs, k, U32, solo_max=20_000)
    _check(vqs, k, U32, asc=False, solo_max=20_000)
    _check(vqs, np.full(5_000, 3, dtype=np.uint16), U16)


@pytest.mark.parametrize("limit", [1, 2, 4])
def test_forced_depth_limit_fallback(vqs, limit):
    keys = W.uniform_u64(200_000, 2)
    gst = _check(vqs, keys, U64, depth_limit=limit, gpu_limit=limit, solo_max=20_000)
    assert gst["fallbacks"] >= 1


def test_depth_limit_zero_every_range_falls_back(vqs):
    keys = W.uniform_u32(50_000, 3)
    gst = _check(vqs, keys, U32, depth_limit=0, gpu_limit=-1)
    assert gst["fallbacks"] == 1 and gst["partitions"] == 0


def test_zipf_reaches_depth_limit_like_the_oracle(vqs):
    gst = _check(vqs, W.zipf_u64(1_000_000, 3), U64, seed=3, solo_max=20_000)
    assert gst["fallbacks"] > 0


# ---- segmented --------------------------------------------------------------------------

def _check_segmented(vqs, keys, offsets, kt, asc=True, seed=0, **opts):
    import torch
    want = keys.copy()
    ost = oracle.sort_segmented(want, offsets, kt, ascending=asc, seed=seed, stats=True)
    t = to_gpu(keys)
    off = to_gpu(offsets.astype(np.int64))
    vqs.sort_segmented(t, off, ascending=asc, key_type=kt, seed=seed, **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    assert_stats_equal(ost, vqs.get_stats())


@pytest.mark.parametrize("kt", [U32, U64])
def test_segmented_log_uniform(vqs, kt):
    off = W.segment_offsets(500, seed=12, lo=16, hi=1 << 17)
    keys = W.segmented_keys(off, kt, 13)
    _check_segmented(vqs, keys, off, kt, seed=1)


def test_segmented_empty_and_tiny_segments(vqs):
    lens = np.array([0, 1, 0, 2, 3, 0, 16, 255, 256, 257, 0, 5000, 1, 100_000, 0], dtype=np.int64)
    off = np.zeros(lens.size + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    keys = W.uniform_u64(int(off[-1]), 4)
    _check_segmented(vqs, keys, off, U64, solo_max=20_000)
    _check_segmented(vqs, keys, off, U64, asc=False)


def test_segmented_graph_replay(vqs):
    import torch
    off = W.segment_offsets(300, seed=21, lo=16, hi=1 << 15)
    keys = W.uniform_u32(int(off[-1]), 22)
    want = keys.copy()
    oracle.sort_segmented(want, off, U32)
    t = to_gpu(keys)
    o = to_gpu(off)
    for rep in range(3):
        t.copy_(to_gpu(keys))
        torch.cuda.synchronize()
        vqs.sort_segmented(t, o, key_type=U32, use_graph=1)
        torch.cuda.synchronize()
        assert vqs.last_error_bits() == 0
        np.testing.assert_array_equal(to_host(t), want)


def test_autotune_segmented(vqs, tmp_path):
    """The tuner returns one of its candidates, leaves the caller's keys alone, the
    tuned sort matches the oracle run with the same base-case threshold (so the
    recursion counts agree too), and a cached result is returned as stored."""
    import torch
    off = W.segment_offsets(1500, seed=12, lo=16, hi=1 << 16)
    keys = W.segmented_keys(off, U32, 13)
    t = to_gpu(keys)
    o = to_gpu(off)
    cache = str(tmp_path / "tune.json")
    res = vqs.autotune_segmented(t, o, key_type=U32, max_keys=1_500_000, cache=cache)
    torch.cuda.synchronize()
    assert res["solo_max"] in (0, 1 << 14, 1 << 16, 1 << 18, 1 << 20)
    assert res["base_case"] in (128, 256)
    assert res["local_keys"] in (8192, 4096)
    assert res["level_mode"] in (1, 2)
    assert res["tile_variant"] in (0, 1)
    assert res["best_ms"] > 0
    np.testing.assert_array_equal(to_host(t), keys)          # untouched
    tuned = {k: res[k] for k in vqs.TUNED_FIELDS}
    want = keys.copy()
    ost = oracle.sort_segmented(want, off, U32, nb=tuned["base_case"], stats=True)
    vqs.sort_segmented(t, o, key_type=U32, **tuned)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    assert_stats_equal(ost, vqs.get_stats())
    again = vqs.autotune_segmented(t, o, key_type=U32, max_keys=1_500_000, cache=cache)
    assert again == res


@pytest.mark.parametrize("n", [4, 9, 16, 20, 24])
def test_base_case_every_zero_one_input(vqs, n):
    import torch
    m = 1 << n
    keys = ((np.arange(m, dtype=np.uint64)[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & 1)
    keys = np.ascontiguousarray(keys.astype(np.uint32).reshape(-1))
    off = np.arange(m + 1, dtype=np.int64) * n
    t = to_gpu(keys)
    vqs.sort_segmented(t, to_gpu(off), key_type=U32)
    torch.cuda.synchronize()
    rows = to_host(t).reshape(m, n)
    assert (np.diff(rows.astype(np.int64), axis=1) >= 0).all()
    np.testing.assert_array_equal(rows.sum(axis=1), keys.reshape(m, n).sum(axis=1))


@pytest.mark.parametrize("n", [3, 8, 9])
def test_all_permutations(vqs, n):
    import torch
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.uint64)
    off = np.arange(perms.shape[0] + 1, dtype=np.int64) * n
    t = to_gpu(perms.reshape(-1))
    vqs.sort_segmented(t, to_gpu(off), key_type=U64)
    torch.cuda.synchronize()
    assert (to_host(t).reshape(-1, n) == np.arange(n, dtype=np.uint64)).all()


def test_offset_views_keep_alignment_rules(vqs):
    import torch
    base = W.uniform_u32(100_003, 9)
    t = to_gpu(base)
    sub = t[3:100_001]                # 12 bytes past a 16-byte boundary
    vqs.sort(sub, key_type=U32)
    torch.cuda.synchronize()
    got = to_host(t)
    np.testing.assert_array_equal(got[3:100_001], np.sort(base[3:100_001]))
    np.testing.assert_array_equal(got[:3], base[:3])
    np.testing.assert_array_equal(got[100_001:], base[100_001:])
