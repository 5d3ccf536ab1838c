"""Signed keys, 64-bit keys with 64-bit data, and the stable sort, on the GPU against
the CPU oracle.

  * i16 / i32 / i64 keys (the paper's measurement types): element by element and the
    recursion counters against the oracle's signed instantiation, both orders, sizes
    from one local sort to several device-wide levels, the extreme values included.
  * k64v64 pairs: sorted as the 128-bit key (key, data) as Sec. 2.4 treats them, so
    the output is unique; element by element and counters against the oracle.
  * The stable sort (Sec. 5: a row number appended to the least-significant bits of
    the key): the permutation equals NumPy's stable lexicographic order (a library
    routine) of (key in sort order, input position), the keys equal the permuted
    input, and the counters equal the oracle's sort of the same composite keys.
"""
import numpy as np
import pytest

import oracle
from tests.helpers import F32, F64, U16, U32, U64, assert_stats_equal, to_gpu, to_host

pytestmark = pytest.mark.gpu

I16, I32, I64, K64V64 = 7, 8, 9, 10


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _signed_keys(kt, n, seed, dup=False):
    dt = {I16: np.int16, I32: np.int32, I64: np.int64}[kt]
    info = np.iinfo(dt)
    rng = np.random.default_rng(seed)
    if dup:
        a = rng.integers(-50, 50, n).astype(dt)
    else:
        a = rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
    a[: min(n, 4)] = [info.min, info.max, -1, 0][: min(n, 4)]
    return a


def _check(vqs, keys, kt, asc, **opts):
    import torch
    want = keys.copy()
    ost = oracle.sort(want, kt, ascending=asc, stats=True)
    t = to_gpu(keys)
    vqs.sort(t, ascending=asc, key_type=kt, **opts)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(t), want)
    assert_stats_equal(ost, vqs.get_stats())
    return want


@pytest.mark.parametrize("kt", [I16, I32, I64])
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("n", [1, 200, 5000, 70_001, 1_500_000])
def test_signed_keys(vqs, kt, asc, n):
    print(f"case: signed kt={kt} asc={asc} n={n}", flush=True)
    keys = _signed_keys(kt, n, 100 + n + kt)
    want = _check(vqs, keys, kt, asc)
    ref = np.sort(keys)
    np.testing.assert_array_equal(want, ref if asc else ref[::-1])


@pytest.mark.parametrize("kt", [I16, I32, I64])
def test_signed_keys_heavy_duplicates_and_levels(vqs, kt):
    print(f"case: signed dup kt={kt}", flush=True)
    _check(vqs, _signed_keys(kt, 2_000_000, 7, dup=True), kt, True, solo_max=20_000)
    _check(vqs, _signed_keys(kt, 600_000, 8), kt, False, solo_max=20_000, level_mode=2)


def _kv(n, seed, nkeys):
    rng = np.random.default_rng(seed)
    a = np.empty((n, 2), np.uint64)
    a[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)          # data
    a[:, 1] = rng.integers(0, nkeys, n, dtype=np.uint64)          # key
    return a


@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("n,nkeys", [(3000, 100), (400_000, 2**64 - 1), (1_200_000, 1000)])
def test_k64v64_pairs(vqs, asc, n, nkeys):
    print(f"case: k64v64 asc={asc} n={n}", flush=True)
    kv = _kv(n, n, nkeys)
    want = _check(vqs, kv, K64V64, asc)
    # keys in order, equal keys ordered by their data, the same pairs
    order = np.lexsort((kv[:, 0], kv[:, 1]))
    ref = kv[order] if asc else kv[order][::-1]
    np.testing.assert_array_equal(want, ref)


def _order_form(keys, kt, asc):
    """The keys as unsigned integers in sort order (the plain definition of the order:
    unsigned as is, signed by the sign bit, floats by their total order), complemented
    for descending order."""
    if kt in (F32, F64):
        ut, bits = (np.uint32, 32) if kt == F32 else (np.uint64, 64)
        u = keys.view(ut).astype(np.uint64)
        sign = np.uint64(1) << np.uint64(bits - 1)
        mask = (np.uint64(1) << np.uint64(bits)) - np.uint64(1) if bits < 64 else ~np.uint64(0)
        u = np.where(u & sign, ~u & mask, u | sign)
    elif kt in (I16, I32, I64):
        bits = keys.dtype.itemsize * 8
        u = keys.view({16: np.uint16, 32: np.uint32, 64: np.uint64}[bits]).astype(np.uint64)
        u = u ^ (np.uint64(1) << np.uint64(bits - 1))
    else:
        bits = keys.dtype.itemsize * 8
        u = keys.astype(np.uint64)
    if not asc:
        mask = (np.uint64(1) << np.uint64(bits)) - np.uint64(1) if bits < 64 else ~np.uint64(0)
        u = ~u & mask
    return u


def _stable_keys(kt, n, seed):
    rng = np.random.default_rng(seed)
    if kt == F32:
        return (rng.integers(-40, 40, n) / 4).astype(np.float32) + np.float32(0.0)
    if kt == F64:
        return (rng.integers(-40, 40, n) / 8).astype(np.float64) + 0.0
    if kt in (I16, I32, I64):
        return _signed_keys(kt, n, seed, dup=True)
    dt = {U16: np.uint16, U32: np.uint32, U64: np.uint64}[kt]
    return rng.integers(0, 300, n).astype(dt)


@pytest.mark.parametrize("kt", [U16, U32, U64, F32, F64, I16, I32, I64])
@pytest.mark.parametrize("asc", [True, False])
@pytest.mark.parametrize("n", [5000, 900_000])
def test_stable_sort(vqs, kt, asc, n):
    import torch
    print(f"case: stable kt={kt} asc={asc} n={n}", flush=True)
    keys = _stable_keys(kt, n, 300 + kt + n)
    u = _order_form(keys, kt, asc)
    rows = np.arange(n, dtype=np.uint64)
    perm = np.lexsort((rows, u))                       # stable: equal keys by input position
    # the oracle's sort of the composite keys (Sec. 5), with its recursion counters
    if keys.dtype.itemsize <= 4:
        comp, ckt = (u << np.uint64(32)) | rows, oracle.U64
    else:
        comp, ckt = np.stack([rows, u], axis=1).copy(), oracle.U128
    ost = oracle.sort(comp, ckt, stats=True)
    got_rows_oracle = comp & np.uint64(0xFFFFFFFF) if ckt == oracle.U64 else comp[:, 0]
    np.testing.assert_array_equal(got_rows_oracle.astype(np.int64), perm)
    t = to_gpu(keys)
    _, r = vqs.sort_stable(t, ascending=asc, key_type=kt)
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    np.testing.assert_array_equal(to_host(r), perm)
    np.testing.assert_array_equal(to_host(t), keys[perm])
    assert_stats_equal(ost, vqs.get_stats())


def test_stable_sort_wide_rows_and_no_rows(vqs):
    """64-bit keys take the 128-bit composite; without a rows array the keys still come
    out in stable order (equal keys are bit-identical, so only the keys show)."""
    import torch
    print("case: stable no rows", flush=True)
    keys = _stable_keys(I64, 300_000, 5)
    t = to_gpu(keys)
    _, r = vqs.sort_stable(t, key_type=I64, rows=False)
    torch.cuda.synchronize()
    assert r is None
    np.testing.assert_array_equal(to_host(t), np.sort(keys, kind="stable"))
