"""Pins of the oracle's in-place Partition (Sec. 2.1, the bidirectional scan with
CompressStore; 64-key vectors, four per loop iteration), against facts that do not
come from re-running its own steps:

  * the partition property, the bound and the multiset on many sizes, pivots, types
    and both orders (a store that overwrote an unread key would lose it);
  * closed forms: every key left (the range rotates: remainder, loop blocks, then the
    two held-back blocks), every key right (vector order reversed, the tie rule and
    the remainder move visible), and ranges under two blocks (a stable split);
  * a second formulation: the capacity rule "load the side with less capacity" is
    the same as merging two non-decreasing count sequences (right keys read on the
    left, left keys read on the right) with ties to the left, so each block's step
    is its rank in that merge (searchsorted) instead of a simulation of the loop.
"""
import numpy as np
import pytest

import oracle

B, V = oracle.IP_BLOCK, oracle.IP_LANES
ONE_D = [oracle.U16, oracle.U32, oracle.U64, oracle.F32, oracle.F64, oracle.I32]


def _keys(kt, n, rng, distinct=None):
    dt = oracle._DTYPES[kt]
    if kt in (oracle.F32, oracle.F64):
        a = rng.standard_normal(n).astype(dt)
        if distinct:
            a = np.round(a * distinct).astype(dt)
        return a
    info = np.iinfo(dt)
    hi = info.max if distinct is None else min(info.max, info.min + distinct)
    return rng.integers(info.min, hi, n, dtype=dt, endpoint=True)


def _isleft(a, piv, asc):
    return (a <= piv) if asc else (a >= piv)


def merge_path_reference(keys, isl, ties_left=True):
    """The partition's output from the block order the merge ranks give."""
    n = keys.shape[0]
    out = np.empty_like(keys)
    if n < 2 * B:
        nl = int(isl.sum())
        out[:nl], out[nl:] = keys[isl], keys[~isl]
        return out, nl
    nrem = n % B
    lrem = isl[:nrem]
    lr = int(lrem.sum())
    rr = nrem - lr
    out[:lr], out[n - rr:] = keys[:nrem][lrem], keys[:nrem][~lrem]
    # the main loop's input: the range's last rr keys, moved into the gap, then the rest
    src = np.concatenate([np.arange(n - rr, n), np.arange(nrem, n - rr)])
    mk, ml = keys[src], isl[src]
    m = mk.shape[0] // B
    nl = m - 2                                   # loop blocks 1 .. m-2
    c = ml.reshape(m, B).sum(1)
    P = np.concatenate([[0], np.cumsum(c[1:m - 1])])
    A = B * np.arange(nl) - P[:nl]               # right keys among the first i left blocks
    Bq = P[-1] - P[nl - np.arange(nl)]           # left keys among the last j loop blocks
    sa, sb = ("left", "right") if ties_left else ("right", "left")
    pos_a = np.arange(nl) + np.searchsorted(Bq, A, side=sa)
    pos_b = np.arange(nl) + np.searchsorted(A, Bq, side=sb)
    steps = sorted([(pos_a[i], 1 + i) for i in range(nl) if pos_a[i] < nl] +
                   [(pos_b[j], nl - j) for j in range(nl) if pos_b[j] < nl])
    assert [s for s, _ in steps] == list(range(nl))
    wl, wr = lr, n - rr
    for blk in [b for _, b in steps] + [0, m - 1]:
        for v in range(B // V):
            sl = slice(blk * B + v * V, blk * B + (v + 1) * V)
            kk, ll = mk[sl], ml[sl]
            k = int(ll.sum())
            out[wl:wl + k] = kk[ll]
            wl += k
            wr -= V - k
            out[wr:wr + V - k] = kk[~ll]
    assert wl == wr
    return out, wl


SIZES = [0, 1, 63, 255, 256, 300, 511, 512, 513, 767, 768, 1024, 1279, 5000, 65_536, 100_003]


@pytest.mark.parametrize("kt", ONE_D)
@pytest.mark.parametrize("asc", [True, False])
def test_inplace_partition_is_a_partition(kt, asc):
    rng = np.random.default_rng(40 + kt)
    for n in SIZES:
        for distinct in (None, 3):
            a = _keys(kt, n, rng, distinct)
            if n == 0:
                assert oracle.partition_inplace(a.copy(), 0, 0, 0, kt, asc) == 0
                continue
            piv = a[rng.integers(0, n)]
            k = a.copy()
            bound = oracle.partition_inplace(k, 0, n, piv, kt, asc)
            isl = _isleft(a, piv, asc)
            assert bound == int(isl.sum())
            assert _isleft(k[:bound], piv, asc).all() and not _isleft(k[bound:], piv, asc).any()
            np.testing.assert_array_equal(np.sort(k), np.sort(a))


def test_inplace_partition_u128_is_a_partition():
    rng = np.random.default_rng(9)
    for n in (600, 3000):
        a = np.empty((n, 2), np.uint64)
        a[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)
        a[:, 1] = rng.integers(0, 3, n, dtype=np.uint64)
        piv = a[n // 3].copy()
        k = a.copy()
        bound = oracle.partition_inplace(k, 0, n, piv, oracle.U128, True)
        ints = [(int(h) << 64) | int(l) for l, h in a]
        pv = (int(piv[1]) << 64) | int(piv[0])
        isl = np.array([v <= pv for v in ints])
        want, wb = merge_path_reference(np.arange(n), isl)
        assert bound == wb
        np.testing.assert_array_equal(k, a[want])


def test_inplace_only_touches_its_range():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2**32, 9000, dtype=np.uint32)
    k = a.copy()
    bound = oracle.partition_inplace(k, 1234, 7777, a[5000], oracle.U32, True)
    np.testing.assert_array_equal(k[:1234], a[:1234])
    np.testing.assert_array_equal(k[7777:], a[7777:])
    want, wb = merge_path_reference(a[1234:7777], a[1234:7777] <= a[5000])
    assert bound == 1234 + wb
    np.testing.assert_array_equal(k[1234:7777], want)


@pytest.mark.parametrize("n", [512, 513, 1000, 4096, 4097 + 255])
def test_inplace_all_left_rotates_the_blocks(n):
    """Pivot = the largest key: the capacity rule always reads on the left (the right
    side never gains capacity), so the loop blocks come out in order, followed by the
    held-back first and last blocks; the remainder stays in front."""
    a = np.arange(1, n + 1, dtype=np.uint64)[np.random.default_rng(n).permutation(n)]
    k = a.copy()
    assert oracle.partition_inplace(k, 0, n, a.max(), oracle.U64, True) == n
    r = n % B
    main = a[r:]
    want = np.concatenate([a[:r], main[B:-B], main[:B], main[-B:]])
    np.testing.assert_array_equal(k, want)


@pytest.mark.parametrize("n", [512, 700, 1024, 2048 + 100])
def test_inplace_all_right_reverses_the_vectors(n):
    """Pivot before every key: the remainder (all right) goes to the end in order,
    the range's last keys move to the front; the loop reads the first loop block (a
    tie at the start goes left), then only right blocks from the end; every
    vector's keys land just below the previous vector's, so the main region holds
    the vectors of the read sequence (loop blocks, first, last) in reverse order."""
    a = np.arange(10, 10 + n, dtype=np.uint32)[np.random.default_rng(n).permutation(n)]
    k = a.copy()
    assert oracle.partition_inplace(k, 0, n, np.uint32(0), oracle.U32, True) == 0
    r = n % B
    main = np.concatenate([a[n - r:], a[r:n - r]])
    m = main.size // B
    seq = ([1] + list(range(m - 2, 1, -1)) if m > 2 else []) + [0, m - 1]
    vecs = [main[blk * B + v * V: blk * B + (v + 1) * V] for blk in seq for v in range(B // V)]
    want = np.concatenate([np.concatenate(vecs[::-1]), a[:r]])
    np.testing.assert_array_equal(k, want)


@pytest.mark.parametrize("n", [2, 100, 256, 511])
def test_inplace_small_range_is_a_stable_split(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 50, n, dtype=np.uint16)
    for asc in (True, False):
        k = a.copy()
        piv = a[n // 2]
        isl = _isleft(a, piv, asc)
        assert oracle.partition_inplace(k, 0, n, piv, oracle.U16, asc) == int(isl.sum())
        np.testing.assert_array_equal(k, np.concatenate([a[isl], a[~isl]]))


@pytest.mark.parametrize("kt", [oracle.U64, oracle.F32, oracle.U16])
@pytest.mark.parametrize("asc", [True, False])
def test_inplace_matches_the_merge_path_formulation(kt, asc):
    rng = np.random.default_rng(70 + kt + asc)
    for t in range(60):
        n = int(rng.integers(2 * B, 30_000))
        a = _keys(kt, n, rng, distinct=None if t % 2 else 200)
        if t % 3 == 0:
            # blocks of very different left densities: long runs on one side
            dens = np.repeat(rng.random(n // 97 + 1), 97)[:n]
            lo_hi = np.sort(a[rng.integers(0, n, 2)])
            a = np.where(rng.random(n) < dens, lo_hi[0], lo_hi[1]).astype(a.dtype)
        piv = a[rng.integers(0, n)]
        k = a.copy()
        bound = oracle.partition_inplace(k, 0, n, piv, kt, asc)
        want, wb = merge_path_reference(a, _isleft(a, piv, asc))
        assert bound == wb
        np.testing.assert_array_equal(k, want)


def test_a_tie_to_the_right_is_caught():
    """The first loop iteration always meets a tie (both capacities equal); reading
    the right side there instead of the left gives another order."""
    rng = np.random.default_rng(1)
    a = rng.integers(0, 2**64, 4096, dtype=np.uint64)
    piv = a[7]
    k = a.copy()
    oracle.partition_inplace(k, 0, a.size, piv, oracle.U64, True)
    other, _ = merge_path_reference(a, a <= piv, ties_left=False)
    assert not np.array_equal(k, other)


@pytest.mark.parametrize("kt", [oracle.U64, oracle.U32, oracle.U128, oracle.F64, oracle.I16])
@pytest.mark.parametrize("asc", [True, False])
def test_sort_with_the_inplace_partition(kt, asc):
    rng = np.random.default_rng(5 + kt)
    for n in (0, 100, 777, 20_000, 200_000):
        if kt == oracle.U128:
            a = np.empty((n, 2), np.uint64)
            a[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)
            a[:, 1] = rng.integers(0, 4, n, dtype=np.uint64)
        else:
            a = _keys(kt, n, rng, distinct=None if n % 2 else 1000)
        k = a.copy()
        st = oracle.sort(k, kt, asc, stats=True, inplace=True)
        w = a.copy()
        oracle.sort(w, kt, asc)                 # the out-of-place sort: same sorted order
        np.testing.assert_array_equal(k, w)
        if n > 100:
            assert st["partitions"] > 0


def test_inplace_recursion_differs_from_the_out_of_place_one():
    """The two Partitions leave the sides in different orders, so later pivots (and
    the recursion counters) differ while the sorted output does not."""
    a = np.random.default_rng(2).integers(0, 2**64, 200_000, dtype=np.uint64)
    k1, k2 = a.copy(), a.copy()
    s1 = oracle.sort(k1, oracle.U64, stats=True, inplace=True)
    s2 = oracle.sort(k2, oracle.U64, stats=True)
    np.testing.assert_array_equal(k1, k2)
    assert s1 != s2
