"""Pins of the CPU oracle against facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: library sorts
(np.sort, Python's sorted on ints), numpy's SFC64, exhaustive 0-1 inputs, closed
forms, special cases and the paper's worked examples (tests/golden/).
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2205_05982_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TYPES = [oracle.U16, oracle.U32, oracle.U64, oracle.U128, oracle.F32, oracle.F64]


def _read_pairs(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            a, b = line.split()
            out.append((int(a), int(b)))
    return out


def _random_keys(kt, n, seed):
    rng = np.random.default_rng(seed)
    if kt == oracle.U16:
        return rng.integers(0, 2**16, n, dtype=np.uint16)
    if kt == oracle.U32:
        return rng.integers(0, 2**32, n, dtype=np.uint32)
    if kt == oracle.U64:
        return rng.integers(0, 2**64, n, dtype=np.uint64)
    if kt == oracle.U128:
        k = np.empty((n, 2), np.uint64)
        k[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)
        k[:, 1] = rng.integers(0, 4, n, dtype=np.uint64)   # many equal high words
        return k
    if kt == oracle.F32:
        a = rng.standard_normal(n, dtype=np.float32) * 1e3
        a[a == 0] = 0.0
        return a
    a = rng.standard_normal(n) * 1e-3
    a[a == 0] = 0.0
    return a


def _expected(keys, kt, asc):
    if kt == oracle.U128:
        ints = sorted(((int(h) << 64) | int(l) for l, h in keys), reverse=not asc)
        return np.array([[v & (2**64 - 1), v >> 64] for v in ints], dtype=np.uint64).reshape(-1, 2)
    s = np.sort(keys, kind="stable")
    return s if asc else s[::-1].copy()


# ---- final output: the plain definition -------------------------------------------

@pytest.mark.parametrize("kt", TYPES)
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("n", [0, 1, 2, 17, 255, 256, 257, 1000, 4096, 50_000])
def test_sort_equals_library_sort(kt, asc, n):
    keys = _random_keys(kt, n, seed=1000 + n + kt)
    got = keys.copy()
    oracle.sort(got, kt, ascending=asc, seed=7)
    np.testing.assert_array_equal(got, _expected(keys, kt, asc))


@pytest.mark.parametrize("dist", W.C2_DISTRIBUTIONS)
def test_sort_c2_distributions_small(dist):
    keys = W.c2(dist, 200_000)
    got = keys.copy()
    st = oracle.sort(got, oracle.U64, seed=3, stats=True)
    np.testing.assert_array_equal(got, np.sort(keys))
    if dist == "zipf":
        # A heavy value that is the maximum of its range makes the partition
        # degenerate; the paper's rule (pivot := first key in sort order) then peels
        # one distinct value per re-partition, so such ranges reach the depth limit.
        assert st["heapsorts"] > 0 and st["degenerate"] > 0
    else:
        assert st["heapsorts"] == 0      # random sampling is not fooled by these inputs


def test_c1_uniform_u32_full_size():
    keys = W.uniform_u32(1_000_000, 1)
    got = keys.copy()
    oracle.sort(got, oracle.U32, seed=0)
    np.testing.assert_array_equal(got, np.sort(keys))


def test_descending_is_reverse_of_ascending():
    keys = W.zipf_u64(100_000, 3)
    a, d = keys.copy(), keys.copy()
    oracle.sort(a, oracle.U64, True)
    oracle.sort(d, oracle.U64, False)
    np.testing.assert_array_equal(d, a[::-1])


def test_u16_counts_match_counting_sort():
    keys = W.uniform_u16(300_000, 10)
    got = keys.copy()
    oracle.sort(got, oracle.U16)
    counts = np.bincount(keys, minlength=65536)
    np.testing.assert_array_equal(got, np.repeat(np.arange(65536, dtype=np.uint16), counts))


def test_segmented_sorts_each_segment():
    off = W.segment_offsets(300, seed=12, lo=16, hi=5000)
    keys = W.uniform_u32(int(off[-1]), 13)
    got = keys.copy()
    oracle.sort_segmented(got, off, oracle.U32)
    for i in range(off.size - 1):
        np.testing.assert_array_equal(got[off[i]:off[i + 1]], np.sort(keys[off[i]:off[i + 1]]))


# ---- networks: 0-1 principle and the paper's worked examples -------------------------

def _zero_one_sorts(net, n):
    x = ((np.arange(1 << n, dtype=np.int64)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    for a, b in net:
        lo = np.minimum(x[:, a], x[:, b])
        x[:, b] = np.maximum(x[:, a], x[:, b])
        x[:, a] = lo
    return bool((np.diff(x.astype(np.int8), axis=1) >= 0).all())


def test_green16_is_a_60_module_sorting_network():
    net = oracle.green16()
    assert len(net) == 60                       # Sec. 3: Green's network, 60 modules
    assert all(0 <= a < b < 16 for a, b in net)
    assert _zero_one_sorts(net, 16)             # all 2^16 0-1 inputs
    # ten layers: greedy layering of the listed order
    layers, used = 1, set()
    for a, b in net:
        if a in used or b in used:
            layers, used = layers + 1, set()
        used |= {a, b}
    assert layers == 10


def test_green16_is_minimal_sized_against_a_dropped_module():
    net = oracle.green16()
    for drop in range(len(net)):
        assert not _zero_one_sorts(net[:drop] + net[drop + 1:], 16)


def test_merge8_equals_fig2():
    fig2 = [(a - 1, b - 1) for a, b in _read_pairs("fig2_merge8.txt")]
    assert oracle.merge_network(8) == fig2


@pytest.mark.parametrize("length", [8, 16, 32, 64, 128, 256])
def test_merge_network_merges_all_sorted_zero_one_pairs(length):
    net = np.array(oracle.merge_network(length), dtype=np.int64)
    half = length // 2
    # 0-1 principle for merging networks: every pair of sorted 0-1 halves
    rows = []
    for z1 in range(half + 1):
        for z2 in range(half + 1):
            rows.append(np.r_[np.zeros(z1), np.ones(half - z1), np.zeros(z2), np.ones(half - z2)])
    x = np.array(rows, dtype=np.uint8)
    for a, b in net:
        lo = np.minimum(x[:, a], x[:, b])
        x[:, b] = np.maximum(x[:, a], x[:, b])
        x[:, a] = lo
    assert (np.diff(x.astype(np.int8), axis=1) >= 0).all()
    assert len(net) == half * int(math.log2(length))


def test_med3_network_fixture_and_exhaustive():
    assert _read_pairs("med3_network.txt") == [(0, 2), (0, 1), (1, 2)]
    for a, b, c in itertools.product(range(3), repeat=3):
        assert oracle.med3_u64(a, b, c, True) == sorted((a, b, c))[1]
        assert oracle.med3_u64(a, b, c, False) == sorted((a, b, c))[1]


@pytest.mark.parametrize("n", list(range(1, 21)))
def test_basecase_all_zero_one_inputs(n):
    # every 0-1 input of length n, each sorted by BaseCase (segments of n <= nb keys)
    m = 1 << n
    keys = ((np.arange(m, dtype=np.uint64)[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & 1)
    keys = np.ascontiguousarray(keys.astype(np.uint32).reshape(-1))
    off = np.arange(m + 1, dtype=np.int64) * n
    st = oracle.sort_segmented(keys, off, oracle.U32, nb=256, stats=True)
    rows = keys.reshape(m, n)
    assert (np.diff(rows.astype(np.int64), axis=1) >= 0).all()
    assert (rows.sum(axis=1) == np.array([bin(i).count("1") for i in range(m)])).all()
    assert st["partitions"] == 0 and st["basecases"] == m


def _bitsliced_inputs(ncells, nfree, word0, nwords):
    """Wires of 64 * nwords 0-1 inputs, bitsliced: input number i = 64 * (word0 + w) + b
    sits in bit b of word w, and wire k carries bit k of i (k < nfree); the other wires
    are the padding, all ones."""
    lanes = np.arange(64, dtype=np.uint64)
    wires = []
    words = np.arange(word0, word0 + nwords, dtype=np.uint64)
    for k in range(ncells):
        if k >= nfree:
            wires.append(np.full(nwords, ~np.uint64(0)))
        elif k < 6:
            pat = np.uint64(0)
            for b in lanes[((lanes >> np.uint64(k)) & np.uint64(1)) == 1]:
                pat |= np.uint64(1) << b
            wires.append(np.full(nwords, pat))
        else:
            wires.append(np.where((words >> np.uint64(k - 6)) & np.uint64(1), ~np.uint64(0), np.uint64(0)))
    return wires


def _run_network_bitsliced(pairs, wires):
    for a, b in pairs:
        lo = wires[a] & wires[b]
        wires[b] = wires[a] | wires[b]
        wires[a] = lo
    return wires


@pytest.fixture(scope="module")
def zero_one(tmp_path_factory):
    """The bitsliced exhaustive checker (tests/zero_one_check.c), built with gcc."""
    import ctypes
    import subprocess
    out = tmp_path_factory.mktemp("zo") / "libzo.so"
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zero_one_check.c")
    subprocess.run(["gcc", "-O3", "-march=native", "-shared", "-fPIC", "-o", str(out), src], check=True)
    L = ctypes.CDLL(str(out))
    L.zero_one_check.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.zero_one_check.restype = ctypes.c_int64

    def check(pairs, order, cells, nfree):
        p = np.ascontiguousarray(pairs, dtype=np.uint32)
        o = np.ascontiguousarray(order, dtype=np.uint32)
        return int(L.zero_one_check(p.ctypes.data, p.shape[0], o.ctypes.data, cells, nfree))
    return check


@pytest.mark.parametrize("n", [16, 32])
def test_basecase_network_sorts_every_zero_one_input(zero_one, n):
    """0-1 principle, exhaustively: the module list BaseCase applies (one column for
    n <= 16, two columns and one merge for n <= 32) sorts all 2^n 0-1 inputs of its
    cells, so every input of up to n keys (the rest padded with the last value) is
    sorted.  Bitsliced, 64 inputs per word: 2^32 inputs for the two-column network."""
    pairs, order, cells = oracle.basecase_network(n)
    assert cells == n
    assert zero_one(pairs, order, cells, n) == -1


def test_zero_one_checker_finds_a_dropped_module(zero_one):
    """The checker is not vacuous: the two-column network without one of its merge
    modules, or with two output positions swapped, fails it."""
    pairs, order, cells = oracle.basecase_network(32)
    assert zero_one(np.delete(pairs, 150, axis=0), order, cells, 32) >= 0
    bad = order.copy()
    bad[[3, 20]] = bad[[20, 3]]
    assert zero_one(pairs, bad, cells, 20) >= 0


@pytest.mark.parametrize("n", [33, 64, 100, 128, 256, 1000])
def test_basecase_network_random_zero_one_inputs(n):
    """Wider base cases on 2^20 random 0-1 inputs each (bitsliced); every merge stage
    they are built from is exhaustively checked above by the 0-1 principle for merging
    networks, and the columns by Green-16's."""
    pairs, order, cells = oracle.basecase_network(n)
    rng = np.random.default_rng(n)
    nwords = 1 << 14
    wires = [rng.integers(0, 2**64, nwords, dtype=np.uint64) if k < n else np.full(nwords, ~np.uint64(0))
             for k in range(cells)]
    ones = sum(np.array([bin(int(x)).count("1") for x in w[:64]]) for w in wires)
    wires = _run_network_bitsliced(pairs, wires)
    out = [wires[int(c)] for c in order]
    for k in range(cells - 1):
        assert not (out[k] & ~out[k + 1]).any(), (n, k)
    assert (sum(np.array([bin(int(x)).count("1") for x in w[:64]]) for w in out) == ones).all()


def test_basecase_uses_its_network():
    """BaseCase on random keys equals its module list applied to the padded buffer."""
    rng = np.random.default_rng(3)
    for n in (2, 15, 16, 17, 31, 32, 33, 200, 256, 1000):
        keys = rng.integers(0, 1000, n).astype(np.uint32)
        got = keys.copy()
        oracle.basecase(got, oracle.U32)
        pairs, order, cells = oracle.basecase_network(n)
        buf = np.full(cells, 0xFFFFFFFF, dtype=np.uint32)
        buf[:n] = keys
        for a, b in pairs:
            x, y = buf[a], buf[b]
            buf[a], buf[b] = min(x, y), max(x, y)
        np.testing.assert_array_equal(got, buf[order[:n]])
        np.testing.assert_array_equal(got, np.sort(keys))


@pytest.mark.parametrize("n", [2, 3, 5, 8, 9])
def test_basecase_all_permutations(n):
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.uint64)
    keys = np.ascontiguousarray(perms.reshape(-1))
    off = np.arange(perms.shape[0] + 1, dtype=np.int64) * n
    oracle.sort_segmented(keys, off, oracle.U64, nb=256)
    assert (keys.reshape(-1, n) == np.arange(n, dtype=np.uint64)).all()


@pytest.mark.parametrize("kt", TYPES)
@pytest.mark.parametrize("asc", [True, False])
def test_basecase_every_size_with_padding(kt, asc):
    for n in range(0, 257):
        keys = _random_keys(kt, n, seed=n)
        got = keys.copy()
        oracle.basecase(got, kt, asc)
        np.testing.assert_array_equal(got, _expected(keys, kt, asc))


def test_basecase_with_extreme_keys_keeps_padding_out():
    # keys equal to the padding value must not be confused with padding
    keys = np.array([2**64 - 1, 0, 2**64 - 1, 5, 7] * 20, dtype=np.uint64)
    got = keys.copy()
    oracle.basecase(got, oracle.U64, True)
    np.testing.assert_array_equal(got, np.sort(keys))
    got = keys.copy()
    oracle.basecase(got, oracle.U64, False)
    np.testing.assert_array_equal(got, np.sort(keys)[::-1])


# ---- random numbers and sampling -----------------------------------------------------

def test_sfc64_matches_numpy():
    for state in ([1, 2, 3, 4], [0xDEADBEEF, 2**63 + 5, 12345678901234567, 1],
                  [2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1]):
        bg = np.random.SFC64()
        bg.state = {"bit_generator": "SFC64",
                    "state": {"state": np.array(state, dtype=np.uint64)},
                    "has_uint32": 0, "uinteger": 0}
        np.testing.assert_array_equal(oracle.sfc64_raw(state, 1000), bg.random_raw(1000))


def test_splitmix64_known_answers():
    # Published reference outputs of SplitMix64 started from state 0.
    assert oracle.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_multiply_shift_offsets_closed_form():
    for rng_ in (1, 3, 7, 1000, 2**24, 2**31 + 11, 2**32 - 1):
        for v in sorted({0, 1, rng_ // 2, rng_ - 1} & set(range(rng_)) if rng_ < 8 else {0, 1, rng_ // 2, rng_ - 1}):
            lo = -((-v << 32) // rng_)               # ceil(v * 2^32 / range): first draw giving v
            assert oracle.multiply_shift(lo, rng_) == v
            if lo > 0:
                assert oracle.multiply_shift(lo - 1, rng_) == v - 1
        assert oracle.multiply_shift(2**32 - 1, rng_) == rng_ - 1
    # bias: each value is hit floor or ceil of 2^32/range times; relative spread < range/2^32
    r = 2**24
    counts = {}
    for v in (0, 5, r - 1):
        first = -((-v << 32) // r)
        nxt = -((-(v + 1) << 32) // r)
        counts[v] = nxt - first
    assert set(counts.values()) <= {2**32 // r, 2**32 // r + 1}


def _pivot_independent(keys, b, e, w, seed, asc=True):
    """ChoosePivot recomputed from the description of Sec. 2.2 with numpy's SFC64
    for the draws and numpy sorts for the medians."""
    bg = np.random.SFC64()
    bg.state = {"bit_generator": "SFC64", "state": {"state": oracle.seg_rng_state(seed, b, e)},
                "has_uint32": 0, "uinteger": 0}
    draws = bg.random_raw(5)
    halves = []
    for d in draws.tolist():
        halves += [d & 0xFFFFFFFF, d >> 32]
    nch = (e - b) // w
    offs = [(u * nch) >> 32 for u in halves[:9]]
    chunks = np.array([keys[b + o * w: b + o * w + w] for o in offs])
    med = lambda x, y, z: np.sort(np.stack([x, y, z]), axis=0)[1]
    cur = np.concatenate([med(chunks[3 * g], chunks[3 * g + 1], chunks[3 * g + 2]) for g in range(3)])
    while cur.size >= 3:
        out, i = [], 0
        while i + 3 * w <= cur.size:
            out.append(med(cur[i:i + w], cur[i + w:i + 2 * w], cur[i + 2 * w:i + 3 * w]))
            i += 3 * w
        while i + 3 <= cur.size:
            out.append(med(cur[i:i + 1], cur[i + 1:i + 2], cur[i + 2:i + 3]))
            i += 3
        cur = np.concatenate(out)
    return cur[0]


@pytest.mark.parametrize("kt,w", [(oracle.U16, 32), (oracle.U32, 16), (oracle.U64, 8), (oracle.F64, 8)])
def test_choose_pivot_matches_independent_recomputation(kt, w):
    keys = _random_keys(kt, 20_000, seed=kt)
    for b, e in [(0, 20_000), (100, 5_000), (3, 3 + 9 * w), (777, 20_000)]:
        for seed in (0, 1, 2**40 + 3):
            p = oracle.choose_pivot(keys, b, e, kt, True, seed)
            assert p == _pivot_independent(keys, b, e, w, seed)
            assert p in keys[b:e]


# Chunk i of the nine sampled chunks holds BASE[i] + pi(j) in lane j.  The paper's
# grouping takes lanewise medians of chunks (0,1,2), (3,4,5), (6,7,8): bases
# med(100,200,900) = 200, med(300,800,400) = 400, med(700,600,500) = 600, then
# the first reduction round's lanewise median of those three gives 400 + pi(j) in
# lane j.  (Grouping chunks (0,3,6), (1,4,7), (2,5,8) instead would give 500 + pi(j).)
# The remaining rounds take consecutive triples of the W values 400 + pi(0..W-1),
# dropping 0..2 leftovers, until fewer than three remain; worked by hand for the
# identity lane order and for the reversed one (pi(j) = W - 1 - j):
#   W = 8  (u64, f64):  identity 400..407 -> 401, 404 -> 401;
#                       reversed 407..400 -> 406, 403 -> 406
#   W = 16 (u32, f32):  identity -> 401, 404, 407, 410, 413 -> 404;
#                       reversed -> 414, 411, 408, 405, 402 -> 411
#   W = 32 (u16):       identity -> 401, 404, ..., 428 -> 404, 413, 422 -> 413;
#                       reversed -> 430, 427, ..., 403 -> 427, 418, 409 -> 418
#   W = 4  (u128):      identity 400..403 -> 401; reversed 403..400 -> 402
BASE = [100, 200, 900, 300, 800, 400, 700, 600, 500]
PIVOT_BY_HAND = {8: (401, 406), 16: (404, 411), 32: (413, 418), 4: (401, 402)}


@pytest.mark.parametrize("kt,w", [(oracle.U16, 32), (oracle.U32, 16), (oracle.U64, 8), (oracle.U128, 4),
                                  (oracle.F32, 16), (oracle.F64, 8)])
@pytest.mark.parametrize("reverse", [False, True])
def test_pivot_reduction_grouping_on_structured_chunks(kt, w, reverse):
    """ChoosePivot (Sec. 2.2) on keys whose nine sampled chunks are filled so that the
    chunk grouping, the lanewise reduction and the leftover rule each decide the
    pivot; the expected pivots are worked out by hand above.  The chunk positions come
    from the offset generator pinned against NumPy's SFC64."""
    n = 200 * w
    b, e = 37 * w, n - 5          # a range not starting at 0, with a ragged tail
    seed = next(s for s in range(1000)
                if len(set(oracle.pivot_offsets(s, b, e, w).tolist())) == 9)
    offs = oracle.pivot_offsets(seed, b, e, w)
    lane = np.arange(w)[::-1] if reverse else np.arange(w)
    dt = {oracle.U16: np.uint16, oracle.U32: np.uint32, oracle.U64: np.uint64,
          oracle.F32: np.float32, oracle.F64: np.float64}.get(kt, np.uint64)
    if kt == oracle.U128:
        keys = np.zeros((n, 2), np.uint64)
        keys[:, 0] = np.random.default_rng(5).integers(0, 2**64, n, dtype=np.uint64)   # low words vary
        keys[:, 1] = 50
        for i in range(9):
            c0 = b + int(offs[i]) * w
            keys[c0:c0 + w, 1] = BASE[i] + lane
    else:
        keys = np.full(n, 50, dtype=dt)
        for i in range(9):
            c0 = b + int(offs[i]) * w
            keys[c0:c0 + w] = (BASE[i] + lane).astype(dt)
    want = PIVOT_BY_HAND[w][1 if reverse else 0]
    for asc in (True, False):
        p = oracle.choose_pivot(keys, b, e, kt, asc, seed)
        got = int(p[1]) if kt == oracle.U128 else int(p)
        assert got == want, (kt, reverse, asc, got, want)


def test_pivot_is_central_on_uniform_data():
    keys = W.uniform_u64(1_000_000, 2)
    ranks = []
    srt = np.sort(keys)
    for s in range(200):
        p = oracle.choose_pivot(keys, 0, keys.size, oracle.U64, True, s)
        ranks.append(np.searchsorted(srt, p) / keys.size)
    ranks = np.array(ranks)
    assert abs(np.median(ranks) - 0.5) < 0.05
    assert ranks.min() > 0.15 and ranks.max() < 0.85


def test_pivot_of_constant_range_is_the_constant():
    keys = np.full(1000, 42, dtype=np.uint32)
    assert oracle.choose_pivot(keys, 0, 1000, oracle.U32, True, 5) == 42


def test_pivot_sorted_range_descending_order():
    keys = np.arange(10_000, dtype=np.uint64)
    pa = oracle.choose_pivot(keys, 0, 10_000, oracle.U64, True, 9)
    pd = oracle.choose_pivot(keys, 0, 10_000, oracle.U64, False, 9)
    assert pa == pd            # the median of three does not depend on the direction


# ---- partition, degenerate path, depth limit -------------------------------------------

@pytest.mark.parametrize("kt", TYPES)
def test_partition_bound_and_sides(kt):
    keys = _random_keys(kt, 5000, seed=3 + kt)
    for asc in (True, False):
        k = keys.copy()
        b, e = 123, 4321
        piv = keys[2000]
        bound = oracle.partition(k, b, e, piv, kt, asc)
        seg = keys[b:e]
        if kt == oracle.U128:
            ints = [(int(h) << 64) | int(l) for l, h in seg]
            pv = (int(piv[1]) << 64) | int(piv[0])
            isleft = np.array([(v <= pv) if asc else (v >= pv) for v in ints])
        else:
            isleft = (seg <= piv) if asc else (seg >= piv)
        assert bound == b + int(isleft.sum())
        np.testing.assert_array_equal(k[b:bound], seg[isleft])          # left: input order
        np.testing.assert_array_equal(k[bound:e], seg[~isleft][::-1])   # right: reverse order
        np.testing.assert_array_equal(k[:b], keys[:b])
        np.testing.assert_array_equal(k[e:], keys[e:])


@pytest.mark.parametrize("kt", TYPES)
def test_partition_at_the_largest_key_leaves_the_range_unchanged(kt):
    """What lets the GPU take a degenerate partition without a pass over the keys:
    with the range's largest key (in sort order) as pivot every key goes left, in
    input order, so the range is exactly as before; and the two parts of any
    partition have as their largest keys the pivot (left) and the range's own
    (right), which is how a range's largest key is known before its partition."""
    keys = _random_keys(kt, 3000, seed=11 + kt)
    for asc in (True, False):
        b, e = 17, 2900
        first, last = oracle.minmax(keys, b, e, kt, asc)
        k = keys.copy()
        assert oracle.partition(k, b, e, last, kt, asc) == e
        np.testing.assert_array_equal(k, keys)
        # a partition at an inner key: the parts' largest keys
        k = keys.copy()
        piv = keys[1000]
        bound = oracle.partition(k, b, e, piv, kt, asc)
        assert b < bound < e
        _, lmax = oracle.minmax(k, b, bound, kt, asc)
        _, rmax = oracle.minmax(k, bound, e, kt, asc)
        np.testing.assert_array_equal(np.asarray(lmax), np.asarray(piv))
        np.testing.assert_array_equal(np.asarray(rmax), np.asarray(last))


def test_all_equal_input_takes_degenerate_path_once():
    keys = np.full(100_000, 7, dtype=np.uint64)
    st = oracle.sort(keys, oracle.U64, stats=True)
    assert st == {**st, "partitions": 1, "degenerate": 1, "all_equal": 1, "basecases": 0}
    assert (keys == 7).all()


def test_two_value_input_repartitions_with_first_key():
    keys = np.array([5] * 30_000 + [9] * 70_000, dtype=np.uint32)
    np.random.default_rng(0).shuffle(keys)
    for asc in (True, False):
        k = keys.copy()
        st = oracle.sort(k, oracle.U32, ascending=asc, stats=True)
        np.testing.assert_array_equal(k, np.sort(keys) if asc else np.sort(keys)[::-1])
        assert st["all_equal"] == 2            # each value ends in one all-equal range
        assert st["degenerate"] >= 2


def test_minmax_first_last():
    keys = W.normal_f32(10_000, 7)
    f, l = oracle.minmax(keys, 10, 9000, oracle.F32, True)
    assert f == keys[10:9000].min() and l == keys[10:9000].max()
    f, l = oracle.minmax(keys, 10, 9000, oracle.F32, False)
    assert f == keys[10:9000].max() and l == keys[10:9000].min()


def test_depth_limit_formula():
    for n in (257, 1000, 2**20, 10**8, 2**33 + 1):
        assert oracle.default_depth_limit(n) == 2 * int(math.floor(math.log2(n))) + 4
    assert oracle.default_depth_limit(2**20) == 44


@pytest.mark.parametrize("limit", [0, 1, 3])
def test_forced_depth_limit_falls_back_to_heapsort(limit):
    keys = W.uniform_u64(50_000, 2)
    got = keys.copy()
    st = oracle.sort(got, oracle.U64, depth_limit=limit, stats=True)
    np.testing.assert_array_equal(got, np.sort(keys))
    assert st["heapsorts"] >= 1
    assert st["max_depth"] <= limit


def test_heapsort_matches_library_sort():
    for kt in TYPES:
        keys = _random_keys(kt, 3000, seed=kt)
        got = keys.copy()
        oracle.heapsort(got, kt, True)
        np.testing.assert_array_equal(got, _expected(keys, kt, True))


def test_planted_partition_mistake_is_caught():
    # A plausible mistake (strict '<' instead of 'not after') changes the bound on
    # a range with keys equal to the pivot; the closed form above catches it.
    keys = np.array([3, 1, 3, 2, 3], dtype=np.uint32)
    k = keys.copy()
    assert oracle.partition(k, 0, 5, 3, oracle.U32, True) == 5
    assert int((keys < 3).sum()) != 5


# ---- adversarial generator self-check ---------------------------------------------------

def _textbook_m3_quicksort_depth(a):
    a = list(a)
    maxd = 0
    stack = [(0, len(a), 1)]
    while stack:
        lo, hi, d = stack.pop()
        while hi - lo > 16:
            maxd = max(maxd, d)
            mid = lo + (hi - lo) // 2
            p = sorted((a[lo], a[mid], a[hi - 1]))[1]
            i, j = lo, hi
            while True:
                while a[i] < p:
                    i += 1
                j -= 1
                while p < a[j]:
                    j -= 1
                if not i < j:
                    break
                a[i], a[j] = a[j], a[i]
                i += 1
            stack.append((i, hi, d + 1))
            hi, d = i, d + 1
    return maxd


def test_median3_killer_drives_textbook_quicksort_linear():
    n = 4000
    k = W.median3_killer_u64(n)
    assert sorted(k.tolist()) == list(range(1, n + 1))
    assert _textbook_m3_quicksort_depth(k.tolist()) > n // 8
    rnd = np.random.default_rng(0).permutation(n) + 1
    assert _textbook_m3_quicksort_depth(rnd.tolist()) < 40
    # the paper's random chunk sampling is not fooled: no Heapsort fallback
    got = W.median3_killer_u64(200_000)
    st = oracle.sort(got, oracle.U64, stats=True)
    assert st["heapsorts"] == 0 and st["max_depth"] < 40
    assert (got == np.arange(1, 200_001, dtype=np.uint64)).all()


# ---- the plain splitter the learned bucket map is measured against --------------------------

U64 = W.U64

def test_plain_split_sizes_partition_the_keys_in_order():
    keys = W.lognormal_mixture_u64(300_000, 15)
    sizes, arranged = oracle.plain_split_sizes(keys, U64, levels=6, return_keys=True)
    assert sizes.sum() == keys.size and sizes.size <= 64 and (sizes > 0).all()
    np.testing.assert_array_equal(np.sort(arranged), np.sort(keys))     # a permutation
    ends = np.cumsum(sizes)
    for i in range(sizes.size - 1):                                      # bucket i before bucket i+1
        assert arranged[ends[i] - sizes[i]:ends[i]].max() <= arranged[ends[i]:ends[i] + sizes[i + 1]].min()


def test_plain_split_one_level_is_one_partition():
    keys = W.uniform_u64(100_000, 2)
    p = oracle.choose_pivot(keys, 0, keys.size, U64)
    sizes = oracle.plain_split_sizes(keys, U64, levels=1)
    np.testing.assert_array_equal(sizes, [np.count_nonzero(keys <= p), np.count_nonzero(keys > p)])


def test_plain_split_degenerate_rule_and_equal_ranges():
    assert oracle.plain_split_sizes(np.full(10_000, 7, np.uint64), U64, levels=8).tolist() == [10_000]
    # two values: whatever the pivot, the round ends with the two runs of equal keys
    keys = np.array([3] * 7_000 + [9] * 5_000, dtype=np.uint64)
    np.random.default_rng(1).shuffle(keys)
    np.testing.assert_array_equal(oracle.plain_split_sizes(keys, U64, levels=1), [7_000, 5_000])


# ---- the secure generator option (Sec. 2.2) ----------------------------------------------

def _rfc8439():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "chacha20_rfc8439.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return {r[0]: r[1:] for r in rows}


def test_chacha20_rfc8439_vectors():
    """The oracle's ChaCha20 quarter round and block function against RFC 8439's
    worked examples (Sec. 2.1.1 and Sec. 2.3.2)."""
    g = _rfc8439()
    q = g["quarter"]
    assert oracle.chacha20_quarter_round(*(int(x, 16) for x in q[:4])) == tuple(int(x, 16) for x in q[5:])
    key = np.frombuffer(bytes(range(32)), dtype="<u4")
    nonce = np.frombuffer(bytes([0, 0, 0, 9, 0, 0, 0, 0x4A, 0, 0, 0, 0]), dtype="<u4")
    np.testing.assert_array_equal(oracle.chacha20_block(key, 1, nonce),
                                  np.array([int(x, 16) for x in g["block"]], dtype=np.uint32))


KEY = np.array([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0, 0x082EFA98,
                0xEC4E6C89], dtype=np.uint32)


def test_chacha20_sampling_offsets_come_from_the_range_block():
    """With a key, the nine chunk offsets of [b, e) are the multiply-shift reductions
    of the first nine words of the ChaCha20 block keyed by it, with block counter =
    low 32 bits of b and nonce = (high 32 bits of b, low and high 32 bits of e)."""
    for b, e, w in [(0, 10_000, 8), (2**33 + 5, 2**33 + 700_000, 16), (123, 2**40, 4)]:
        blk = oracle.chacha20_block(KEY, b & 0xFFFFFFFF, [b >> 32, e & 0xFFFFFFFF, e >> 32])
        nch = (e - b) // w
        want = [oracle.multiply_shift(int(blk[i]), nch) for i in range(9)]
        assert oracle.pivot_offsets(0, b, e, w, rng_key=KEY).tolist() == want
        assert oracle.pivot_offsets(0, b, e, w).tolist() != want    # SFC64 draws differently


@pytest.mark.parametrize("kt", [oracle.U16, oracle.U32, oracle.U64, oracle.U128, oracle.F32, oracle.F64])
def test_sort_with_the_secure_generator(kt):
    """The sort is the plain definition's sorted order with either generator, and the
    pivots (hence the recursion) depend on the key."""
    keys = _random_keys(kt, 60_000, seed=kt + 50)
    a, b = keys.copy(), keys.copy()
    sa = oracle.sort(a, kt, stats=True, rng_key=KEY)
    sb = oracle.sort(b, kt, stats=True)
    np.testing.assert_array_equal(a, b)
    other = KEY.copy()
    other[0] ^= 1
    c = keys.copy()
    sc = oracle.sort(c, kt, stats=True, rng_key=other)
    np.testing.assert_array_equal(c, b)
    assert (sa["keys_partitioned"], sa["basecases"]) != (sb["keys_partitioned"], sb["basecases"]) or \
           (sa["keys_partitioned"], sa["basecases"]) != (sc["keys_partitioned"], sc["basecases"])
