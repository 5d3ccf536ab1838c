"""In-place mode (vqs_options.inplace): every partition in the order of the paper's
in-place bidirectional scan (Sec. 2.1), no scratch array of keys.  Against the
oracle's sort with its in-place Partition (same pivots, so the same recursion): the
output element by element and the eight recursion counters, for every key type and
both orders, in each placement of a partition (the LDS local sort, one workgroup's
partitions through device memory, the device-wide levels), on degenerate inputs,
past the depth limit, in segmented sorts, with the allocation-free entry point, and
at the benchmarked size (1e8 u64).  The workspace is checked to hold no key scratch.
"""
import numpy as np
import pytest

import oracle
from paper_2205_05982_amd import workloads as W
from tests.helpers import F32, F64, U16, U32, U64, U128, assert_stats_equal, random_keys, to_gpu, to_host

pytestmark = pytest.mark.gpu

I32, I64 = 8, 9
KS = {U16: 2, U32: 4, F32: 4, U64: 8, F64: 8, U128: 16, I32: 4, I64: 8}


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _keys(kt, n, seed):
    if kt in (I32, I64):
        dt = np.int32 if kt == I32 else np.int64
        info = np.iinfo(dt)
        return np.random.default_rng(seed).integers(info.min, info.max, n, dtype=dt, endpoint=True)
    return random_keys(kt, n, seed)


def _check(vqs, keys, kt, asc=True, depth_limit=-1, **opts):
    """GPU in-place sort vs the oracle's in-place sort: keys and counters."""
    import torch
    want = keys.copy()
    ost = oracle.sort(want, kt, ascending=asc, stats=True, inplace=True,
                      depth_limit=depth_limit if depth_limit >= 0 else -1)
    t = to_gpu(keys)
    gopts = dict(opts)
    if depth_limit >= 0:
        gopts["depth_limit"] = depth_limit if depth_limit > 0 else -1
    vqs.sort(t, ascending=asc, key_type=kt, inplace=1, **gopts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    gst = vqs.get_stats()
    assert_stats_equal(ost, gst)
    return gst


# placements: default threshold; one workgroup's partitions through device memory
# (solo_max at its in-place maximum); many short device-wide ranges; a small LDS
# capacity (workgroup partitions of ranges under two blocks)
CONFIGS = {"default": {}, "solo_global": {"solo_max": 65536}, "levels": {"solo_max": 1024, "local_keys": 1024},
           "small_lds": {"local_keys": 300, "solo_max": 4096}}


@pytest.mark.parametrize("kt", [U16, U32, U64, U128, F32, F64, I32, I64])
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("config", list(CONFIGS))
def test_inplace_matches_the_oracle(vqs, kt, asc, config):
    for n in (700, 5_000, 70_001, 400_000):
        print(f"case: inplace kt={kt} asc={asc} config={config} n={n}", flush=True)
        st = _check(vqs, _keys(kt, n, 11 * kt + n % 97), kt, asc, **CONFIGS[config])
        if n == 400_000 and config in ("levels", "default"):
            assert st["levels"] >= 1


@pytest.mark.parametrize("kt,asc", [(7, True), (7, False), (10, True), (10, False)])
def test_inplace_i16_and_key_with_data(vqs, kt, asc):
    """i16 keys, and 64-bit keys with 64-bit data (sorted as the 128-bit pair)."""
    rng = np.random.default_rng(20 + kt)
    for n in (900, 60_000, 300_000):
        if kt == 7:
            keys = rng.integers(-2**15, 2**15, n, dtype=np.int16)
        else:
            keys = np.empty((n, 2), np.uint64)
            keys[:, 1] = rng.integers(0, 50, n, dtype=np.uint64)        # the key: many equal
            keys[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)     # the data
        print(f"case: inplace kt={kt} asc={asc} n={n}", flush=True)
        opts = {"solo_max": 4096, "local_keys": 2048} if n > 100_000 else {}
        _check(vqs, keys, kt, asc, **opts)


def test_inplace_stable_sort(vqs):
    """The stable sort on the in-place path: same keys and permutation as without it."""
    import torch
    keys = np.random.default_rng(4).integers(0, 1000, 500_000).astype(np.uint32)
    t1, t2 = to_gpu(keys), to_gpu(keys)
    _, r1 = vqs.sort_stable(t1, key_type=U32)
    _, r2 = vqs.sort_stable(t2, key_type=U32, inplace=1)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t1), to_host(t2))
    np.testing.assert_array_equal(to_host(r1), to_host(r2))
    np.testing.assert_array_equal(to_host(r2), np.argsort(keys, kind="stable"))


@pytest.mark.parametrize("dist", ["all_equal", "two_values", "eight_distinct", "zipf", "sorted", "reverse"])
@pytest.mark.parametrize("config", ["default", "levels"])
def test_inplace_degenerate_and_structured(vqs, dist, config):
    n = 300_000
    rng = np.random.default_rng(5)
    keys = {"all_equal": lambda: np.full(n, 42, np.uint64),
            "two_values": lambda: rng.integers(0, 2, n).astype(np.uint64) * 1000,
            "eight_distinct": lambda: rng.integers(0, 8, n).astype(np.uint64),
            "zipf": lambda: W.zipf_u64(n, 4),
            "sorted": lambda: np.arange(n, dtype=np.uint64),
            "reverse": lambda: np.arange(n, 0, -1).astype(np.uint64)}[dist]()
    print(f"case: inplace {dist} {config}", flush=True)
    st = _check(vqs, keys, U64, **CONFIGS[config])
    if dist in ("all_equal", "two_values", "eight_distinct"):
        assert st["degenerate"] >= 1


@pytest.mark.parametrize("kt,asc", [(U64, True), (F32, False), (U16, True), (U128, False)])
@pytest.mark.parametrize("where", ["lds", "solo_global", "level"])
def test_inplace_bounded_time_sorts(vqs, kt, asc, where):
    """Depth limit 0 and a fallback-mode limit of 0: each range goes to the in-place
    bounded-time sort (the network in LDS, or the bitonic sort through device
    memory), the output equals the oracle's and the fallback is counted once."""
    cap = 32768 // KS[kt]
    n, opts = {"lds": (cap - 5, {}), "solo_global": (6 * cap + 17, {"solo_max": 8 * cap}),
               "level": (20 * cap + 3, {"solo_max": 4 * cap})}[where]
    opts = {k: min(v, 65536) for k, v in opts.items()}
    print(f"case: inplace bounded kt={kt} asc={asc} where={where} n={n}", flush=True)
    st = _check(vqs, random_keys(kt, n, 60 + kt), kt, asc, depth_limit=0,
                fallback_limit=vqs.FALLBACK_LIMIT_ZERO, **opts)
    assert st["fallbacks"] == 1
    if where == "lds":
        assert st["bounded_lds"] == 1
    else:
        assert st["bounded_global"] == 1


@pytest.mark.parametrize("fb", [0, 2])
def test_inplace_past_the_depth_limit(vqs, fb):
    import torch
    n = 400_000
    keys = random_keys(U32, n, 71 + fb)
    want = keys.copy()
    ost = oracle.sort(want, U32, stats=True, inplace=True, depth_limit=2)
    t = to_gpu(keys)
    lim = vqs.FALLBACK_LIMIT_ZERO if fb == 0 else fb
    print(f"case: inplace depth limit 2 fb={fb}", flush=True)
    vqs.sort(t, key_type=U32, inplace=1, depth_limit=2, fallback_limit=lim, solo_max=8192)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    assert_stats_equal(ost, vqs.get_stats())


def test_inplace_segmented(vqs):
    import torch
    rng = np.random.default_rng(8)
    lens = np.concatenate([rng.integers(0, 3000, 300), [0, 1, 511, 512, 100_000, 250_000]])
    rng.shuffle(lens)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    keys = random_keys(U64, int(off[-1]), 9)
    want = keys.copy()
    ost = oracle.sort_segmented(want, off, U64, stats=True, inplace=True)
    t = to_gpu(keys)
    print("case: inplace segmented", flush=True)
    vqs.sort_segmented(t, to_gpu(off), key_type=U64, inplace=1, solo_max=4096)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    assert_stats_equal(ost, vqs.get_stats())


def test_inplace_workspace_has_no_key_scratch(vqs):
    n = 100_000_000
    out_of_place = vqs.workspace_bytes(n, U64)
    inplace = vqs.workspace_bytes(n, U64, inplace=1)
    assert out_of_place >= 8 * n
    # no key array: what is left is the range lists (their worst-case capacities), the
    # saved blocks and the block counts
    assert 0 < inplace <= out_of_place - 8 * n and inplace < 8 * n // 8, (inplace, out_of_place)


def test_inplace_options_rejected(vqs):
    import torch
    t = to_gpu(random_keys(U64, 5000, 1))
    for bad in ({"inplace": 2}, {"inplace": 1, "solo_max": 500}, {"inplace": 1, "solo_max": 1 << 20},
                {"inplace": 1, "method": 1}):
        with pytest.raises(vqs.VqsError) as e:
            vqs.sort(t, key_type=U64, **bad)
        assert e.value.code == -1
    off = to_gpu(np.array([0, 2500, 5000], np.int64))
    with pytest.raises(vqs.VqsError):
        vqs.sort_segmented(t, off, key_type=U64, inplace=1, use_graph=1)
    torch.cuda.synchronize()


def test_inplace_noalloc_fits_what_the_scratch_copy_cannot(vqs):
    """50M u64 keys: the out-of-place workspace (a 400 MB key scratch) exceeds the
    allocation-free entry point's fixed scratch, the in-place one fits."""
    import torch
    n = 50_000_000
    keys = W.c2("uniform", n)
    t = to_gpu(keys)
    with pytest.raises(vqs.VqsError) as e:
        vqs.sort_noalloc(t, key_type=U64)
    assert e.value.code == -7
    print("case: inplace noalloc 5e7", flush=True)
    vqs.sort_noalloc(t, key_type=U64, inplace=1)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    gst = vqs.get_stats()
    got = to_host(t)
    del t
    torch.cuda.empty_cache()
    want = keys.copy()
    ost = oracle.sort(want, U64, stats=True, inplace=True)
    np.testing.assert_array_equal(got, want)
    assert_stats_equal(ost, gst)


def test_inplace_full_size_1e8_u64(vqs):
    """The benchmarked input (1e8 u64 uniform keys) in place: the oracle's in-place
    sort gives the same keys and the same eight recursion counters."""
    import torch
    n = 100_000_000
    keys = W.c2("uniform", n)
    t = to_gpu(keys)
    print("case: inplace 1e8 u64", flush=True)
    vqs.sort(t, key_type=U64, inplace=1)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    gst = vqs.get_stats()
    got = to_host(t)
    del t
    torch.cuda.empty_cache()
    want = keys
    ost = oracle.sort(want, U64, stats=True, inplace=True)
    np.testing.assert_array_equal(got, want)
    assert_stats_equal(ost, gst)
    assert gst["levels"] >= 10
