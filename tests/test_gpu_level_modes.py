"""GPU parity of both placements of the device-wide partition levels.

VQS_LEVEL_LOOKBACK writes each partition contiguously (a tile's offsets come from a
decoupled look-back); VQS_LEVEL_RUNS lets every tile partition into its own interval
and holds a child range as one run per tile of its parent (gathered through a run
table at the next level; a range leaving for the solo kernel is gathered into place
by a copy entry).  The key sequences, and so pivots and recursion, are the same, so
both are checked element by element and counter by counter against the oracle, on
cases that take several levels: every key type, the distributions with degenerate
partitions and fallbacks, the forced depth limit, odd 16-byte offsets, and segments.
"""
import numpy as np
import pytest

import oracle
from paper_2205_05982_amd import workloads as W
from tests.helpers import (F32, F64, U16, U32, U64, U128, assert_stats_equal, random_keys, to_gpu,
                           to_host)

pytestmark = pytest.mark.gpu

MODES = {"lookback": 1, "runs": 2}


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _check(vqs, keys, kt, mode, asc=True, seed=0, depth_limit=-1, gpu_limit=0, **opts):
    import torch
    want = keys.copy()
    ost = oracle.sort(want, kt, ascending=asc, seed=seed, depth_limit=depth_limit, stats=True)
    t = to_gpu(keys)
    vqs.sort(t, ascending=asc, key_type=kt, seed=seed, depth_limit=gpu_limit, level_mode=MODES[mode], **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    gst = vqs.get_stats()
    assert_stats_equal(ost, gst)
    return gst


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("kt", [U16, U32, U64, U128, F32, F64])
@pytest.mark.parametrize("asc", [True, False])
def test_levels_every_type(vqs, mode, kt, asc):
    n = 1_500_000 if kt != U128 else 600_000
    print(f"case: levels mode={mode} kt={kt} asc={asc} n={n}", flush=True)
    gst = _check(vqs, random_keys(kt, n, seed=300 + kt), kt, mode, asc, seed=7, solo_max=20_000)
    assert gst["levels"] >= 3


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dist", W.C2_DISTRIBUTIONS)
def test_levels_distributions(vqs, mode, dist):
    print(f"case: levels mode={mode} C2 {dist} 2e6", flush=True)
    _check(vqs, W.c2(dist, 2_000_000), U64, mode, seed=3, solo_max=30_000)


@pytest.mark.parametrize("mode", list(MODES))
def test_levels_zipf_fallbacks(vqs, mode):
    print(f"case: levels mode={mode} zipf 1e6", flush=True)
    gst = _check(vqs, W.zipf_u64(1_000_000, 3), U64, mode, seed=3, solo_max=20_000)
    assert gst["fallbacks"] > 0


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("limit", [1, 3])
def test_levels_forced_depth_limit(vqs, mode, limit):
    print(f"case: levels mode={mode} depth limit {limit}", flush=True)
    gst = _check(vqs, W.uniform_u64(400_000, 2), U64, mode, depth_limit=limit, gpu_limit=limit,
                 solo_max=20_000)
    assert gst["fallbacks"] >= 1


@pytest.mark.parametrize("mode", list(MODES))
def test_levels_two_values_and_all_equal(vqs, mode):
    k = np.array([5] * 600_000 + [9] * 1_400_000, dtype=np.uint32)
    np.random.default_rng(0).shuffle(k)
    _check(vqs, k, U32, mode, solo_max=20_000)
    _check(vqs, np.full(700_000, 3, dtype=np.uint64), U64, mode, solo_max=20_000)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("shift", [1, 3])
def test_levels_unaligned_views(vqs, mode, shift):
    import torch
    base = W.uniform_u32(1_200_007, 9)
    t = to_gpu(base)
    sub = t[shift:1_200_000 + shift]
    vqs.sort(sub, key_type=U32, solo_max=20_000, level_mode=MODES[mode])
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    got = to_host(t)
    np.testing.assert_array_equal(got[shift:1_200_000 + shift], np.sort(base[shift:1_200_000 + shift]))
    np.testing.assert_array_equal(got[:shift], base[:shift])
    np.testing.assert_array_equal(got[1_200_000 + shift:], base[1_200_000 + shift:])


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("use_graph", [0, 1])
def test_levels_segmented(vqs, mode, use_graph):
    import torch
    off = W.segment_offsets(200, seed=31, lo=16, hi=1 << 18)
    keys = W.segmented_keys(off, U64, 32)
    want = keys.copy()
    ost = oracle.sort_segmented(want, off, U64, seed=2, stats=True)
    t = to_gpu(keys)
    o = to_gpu(off)
    for rep in range(2):
        t.copy_(to_gpu(keys))
        torch.cuda.synchronize()
        vqs.sort_segmented(t, o, key_type=U64, seed=2, solo_max=20_000, use_graph=use_graph,
                           level_mode=MODES[mode])
        torch.cuda.synchronize()
        assert vqs.last_error_bits() == 0
        np.testing.assert_array_equal(to_host(t), want)
    if not use_graph:
        assert_stats_equal(ost, vqs.get_stats())


def test_level_mode_rejects_unknown(vqs):
    import torch
    t = to_gpu(W.uniform_u64(1000, 1))
    with pytest.raises(Exception):
        vqs.sort(t, key_type=U64, level_mode=7)
    torch.cuda.synchronize()


@pytest.mark.parametrize("solo_max", [0, 4096])
def test_runs_more_runs_than_the_tile_list(vqs, solo_max):
    """A child range made of one-key runs: ones with a single zero in every 5120-key
    tile.  The pivot sampled is 1, the partition is degenerate, the repeat with the
    minimum as pivot sends exactly one key per tile left.  Above 2560 tiles, one tile
    of that child touches more runs than its LDS list holds (its keys are then found
    one by one); with the default threshold the child is gathered by a copy entry,
    with a threshold of 4096 by a partition tile.  The tile boundaries are aligned, so
    the array is allocated at a 16-byte boundary."""
    import torch
    tiles = 4300
    n = tiles * 5120
    keys = np.ones(n, dtype=np.uint64)
    keys[np.arange(tiles) * 5120 + 1000] = 0
    opts = {"solo_max": solo_max} if solo_max else {}
    print(f"case: one-key runs, {tiles} tiles, solo_max={solo_max}", flush=True)
    gst = _check(vqs, keys, U64, "runs", **opts)
    assert gst["degenerate"] >= 1


def _heavy(n, kt, frac, top, seed):
    """n keys: a fraction frac of them copies of one value, the others spread values
    below it (top) or above it; shuffled.  u128 keys spread their high word (the low
    word is random below the heavy key's)."""
    rng = np.random.default_rng(seed)
    nh = int(n * frac)
    span = (1 << 15) if kt == U16 else (1 << 20)
    spread = rng.integers(0, span, n - nh)
    heavy = np.full(nh, span if top else 0)
    if not top:
        spread = spread + 1
    k = np.concatenate([heavy, spread])
    perm = rng.permutation(n)
    k = k[perm]
    if kt in (F32, F64):
        return (k.astype(np.float64) * 0.25 - 1000.0).astype(np.float32 if kt == F32 else np.float64)
    if kt == U128:
        lo = rng.integers(0, 1 << 62, n, dtype=np.uint64)
        lo[np.concatenate([np.ones(nh, bool), np.zeros(n - nh, bool)])[perm]] = 7
        return np.stack([lo, k.astype(np.uint64)], axis=1)
    return k.astype({U16: np.uint16, U32: np.uint32}.get(kt, np.uint64))


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("kt", [U16, U32, U64, U128, F32, F64])
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("top", [True, False])
def test_foreseen_degenerate_partitions(vqs, mode, kt, asc, top):
    """The levels foresee a degenerate partition (pivot = the range's known largest key)
    and take it, and the all-equal finding or the repeat with the minimum, without a
    pass over the keys.  A heavy value above spread keys (top) gives long chains of
    them, each peeling the smallest value off, until the depth limit; a heavy value
    below them gives all-equal left parts.  Keys, order and every counter must match the
    oracle, which makes the passes the Alg. 1 way."""
    n = 1_500_000 if kt != U128 else 600_000
    keys = _heavy(n, kt, 0.7, top, 41 + kt)
    print(f"case: foreseen degenerate mode={mode} kt={kt} asc={asc} top={top}", flush=True)
    gst = _check(vqs, keys, kt, mode, asc, seed=5, solo_max=16384)
    assert gst["degenerate"] >= 1


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("use_graph", [0, 1])
def test_foreseen_degenerate_segmented(vqs, mode, use_graph):
    import torch
    off = W.segment_offsets(40, seed=8, lo=1 << 14, hi=1 << 17)
    parts = [_heavy(int(off[i + 1] - off[i]), U64, 0.6, i % 2 == 0, 100 + i) for i in range(len(off) - 1)]
    keys = np.concatenate(parts)
    want = keys.copy()
    ost = oracle.sort_segmented(want, off, U64, seed=4, stats=True)
    t = to_gpu(keys)
    o = to_gpu(off)
    print(f"case: foreseen degenerate segmented mode={mode} graph={use_graph}", flush=True)
    vqs.sort_segmented(t, o, key_type=U64, seed=4, solo_max=4096, use_graph=use_graph, level_mode=MODES[mode])
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    if not use_graph:
        assert_stats_equal(ost, vqs.get_stats())


def test_profile_level_launches_only(vqs):
    """vqs_profile(2) records the device-wide partition launches and nothing else;
    vqs_profile(1) records the other kinds too (planning, solo)."""
    import torch
    keys = to_gpu(W.uniform_u64(2_000_000, 5))
    kinds = {}
    for mode in (2, 1):
        t = keys.clone()
        torch.cuda.synchronize()
        vqs.profile(mode)
        vqs.profile_read()
        vqs.sort(t, key_type=U64, solo_max=20_000)
        torch.cuda.synchronize()
        recs = vqs.profile_read()
        vqs.profile(0)
        kinds[mode] = {r["kind"] for r in recs}
        assert all(r["ms"] >= 0 for r in recs)
    assert kinds[2] == {"level_partition"}
    assert "level_partition" in kinds[1] and "solo" in kinds[1] and len(kinds[1]) >= 3


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("shift", [1, 3])
@pytest.mark.parametrize("asc", [True, False])
def test_foreseen_degenerate_unaligned_view(vqs, mode, shift, asc):
    """Peeling chains and all-equal fills on a view that starts off a 16-byte boundary:
    the keys around the view stay untouched, the view matches the oracle."""
    import torch
    n = 1_200_000
    for top in (True, False):
        inner = _heavy(n, U32, 0.7, top, 77 + shift)
        base = np.concatenate([np.full(shift, 123, np.uint32), inner, np.full(5, 456, np.uint32)])
        t = to_gpu(base)
        want = inner.copy()
        ost = oracle.sort(want, U32, ascending=asc, seed=5, stats=True)
        print(f"case: foreseen degenerate unaligned mode={mode} shift={shift} asc={asc} top={top}", flush=True)
        vqs.sort(t[shift:shift + n], key_type=U32, ascending=asc, seed=5, solo_max=16384, level_mode=MODES[mode])
        torch.cuda.synchronize()
        assert vqs.last_error_bits() == 0
        got = to_host(t)
        np.testing.assert_array_equal(got[shift:shift + n], want)
        np.testing.assert_array_equal(got[:shift], base[:shift])
        np.testing.assert_array_equal(got[shift + n:], base[shift + n:])
        assert_stats_equal(ost, vqs.get_stats())


# ---- the second compiled tile size ------------------------------------------------------

@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("kt", [U16, U32, U64, U128, F32, F64])
@pytest.mark.parametrize("asc", [True, False])
def test_half_tiles_every_type(vqs, mode, kt, asc):
    """Level kernels with half-size tiles (vqs_options.tile_variant = 1): the same key
    sequences, so the same result and counters as the oracle, both placements."""
    n = 1_300_000 if kt != U128 else 500_000
    print(f"case: half tiles mode={mode} kt={kt} asc={asc} n={n}", flush=True)
    gst = _check(vqs, random_keys(kt, n, seed=400 + kt), kt, mode, asc, seed=3, solo_max=20_000, tile_variant=1)
    assert gst["levels"] >= 3


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dist", ["zipf", "8distinct", "m3killer"])
def test_half_tiles_distributions(vqs, mode, dist):
    print(f"case: half tiles dist={dist} mode={mode}", flush=True)
    _check(vqs, W.c2(dist, 800_000), U64, mode, seed=5, solo_max=20_000, tile_variant=1)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_half_tiles_segmented(vqs, use_graph):
    import torch
    print(f"case: half tiles segmented graph={use_graph}", flush=True)
    off = W.segment_offsets(300, seed=41, lo=16, hi=1 << 18)
    keys = W.segmented_keys(off, U32, 42)
    want = keys.copy()
    ost = oracle.sort_segmented(want, off, U32, stats=True)
    t, o = to_gpu(keys), to_gpu(off)
    for rep in range(2):
        t.copy_(to_gpu(keys))
        torch.cuda.synchronize()
        vqs.sort_segmented(t, o, key_type=U32, use_graph=use_graph, tile_variant=1, solo_max=16_384,
                           total_keys=int(off[-1]))
        torch.cuda.synchronize()
        assert vqs.last_error_bits() == 0
        np.testing.assert_array_equal(to_host(t), want)
    if not use_graph:
        assert_stats_equal(ost, vqs.get_stats())
    with pytest.raises(Exception):
        vqs.sort(t, key_type=U32, tile_variant=2)
