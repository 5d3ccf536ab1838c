"""Seeded synthetic inputs shared by the tests, the smoke check and bench.py.

This module holds only input generators (NumPy ``default_rng`` streams); none of
the sorting method's arithmetic lives here.  The paper measures on uniform random
keys only; the other distributions stress the degenerate-partition path, the
pivot sampler and the learned splitter.  Every generator takes the key count, so
tests use the same recipe at small sizes.

Key-type codes follow the library's interface: 1 u16, 2 u32, 3 u64, 4 u128
(uint64 array of shape (n, 2), column 0 the low word), 5 f32, 6 f64.
"""
from __future__ import annotations

import math

import numpy as np

U16, U32, U64, U128, F32, F64 = 1, 2, 3, 4, 5, 6
DTYPE = {U16: np.uint16, U32: np.uint32, U64: np.uint64, U128: np.uint64,
         F32: np.float32, F64: np.float64}
KEY_SIZE = {U16: 2, U32: 4, U64: 8, U128: 16, F32: 4, F64: 8}

_CHUNK = 1 << 24


def uniform_u32(n: int, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 2**32, size=n, dtype=np.uint32)


def uniform_u64(n: int, seed: int = 2) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)


def uniform_u16(n: int, seed: int = 10) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 65536, size=n, dtype=np.uint16)


def _zipf_ranks(rng, n: int, nvalues: int, s: float) -> np.ndarray:
    """Ranks 0..nvalues-1 with P(rank r) proportional to 1/(r+1)^s (inverse CDF)."""
    w = 1.0 / np.arange(1, nvalues + 1, dtype=np.float64) ** s
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(n, dtype=np.int64)
    for i in range(0, n, _CHUNK):
        m = min(_CHUNK, n - i)
        out[i:i + m] = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), nvalues - 1)
    return out


def _distinct_u64(rng, count: int) -> np.ndarray:
    vals = np.unique(rng.integers(0, 2**64, size=count + count // 8 + 16, dtype=np.uint64))
    rng.shuffle(vals)
    assert vals.size >= count
    return vals[:count]


def zipf_u64(n: int, seed: int = 3, s: float = 1.0, nvalues: int = 1 << 20) -> np.ndarray:
    rng = np.random.default_rng(seed)
    table = _distinct_u64(rng, nvalues)
    return table[_zipf_ranks(rng, n, nvalues, s)]


def few_distinct_u64(n: int, seed: int = 4, k: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    vals = _distinct_u64(rng, k)
    return vals[rng.integers(0, k, size=n)]


def sorted_u64(n: int, seed: int = 5) -> np.ndarray:
    return np.sort(uniform_u64(n, seed))


def reverse_u64(n: int, seed: int = 5) -> np.ndarray:
    return sorted_u64(n, seed)[::-1].copy()


def almost_sorted_u64(n: int, seed: int = 5, swap_seed: int = 6, frac: float = 0.01) -> np.ndarray:
    a = sorted_u64(n, seed)
    rng = np.random.default_rng(swap_seed)
    m = int(math.floor(frac * n))
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    for s in range(0, m, _CHUNK):        # swaps applied in order
        ii, jj = i[s:s + _CHUNK], j[s:s + _CHUNK]
        for x, y in zip(ii.tolist(), jj.tolist()):
            a[x], a[y] = a[y], a[x]
    return a


def median3_killer_u64(n: int) -> np.ndarray:
    """Musser's median-of-3 killer permutation of 1..n (n even): odd positions of
    the first half hold 1, 3, 5, ..., each followed by k+i+1 (k = n/2), and the
    second half holds 2, 4, ..., n.  It drives a first/middle/last median-of-3
    quicksort to recursion depth linear in n (checked in the tests)."""
    if n % 2:
        raise ValueError("n must be even")
    k = n // 2
    a = np.empty(n, dtype=np.uint64)
    i = np.arange(1, k + 1, dtype=np.uint64)
    odd = i[(i % 2) == 1]
    a[(odd - 1).astype(np.int64)] = odd
    a[odd.astype(np.int64)] = k + odd
    a[k:] = 2 * i
    return a


def normal_f32(n: int, seed: int = 7) -> np.ndarray:
    a = np.random.default_rng(seed).standard_normal(size=n, dtype=np.float32)
    a[a == 0] = 0.0          # canonical +0.0
    return a


def exponential_f32(n: int, seed: int = 8) -> np.ndarray:
    a = np.random.default_rng(seed).standard_exponential(size=n, dtype=np.float32)
    a[a == 0] = 0.0
    return a


def uniform_f64(n: int, seed: int = 9) -> np.ndarray:
    return np.random.default_rng(seed).random(size=n, dtype=np.float64)


def u128_keys(n: int, seed: int = 11) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty((n, 2), dtype=np.uint64)
    out[:, 1] = rng.integers(0, 2**16, size=n, dtype=np.uint64)    # hi: 2^16 values
    out[:, 0] = rng.integers(0, 2**64, size=n, dtype=np.uint64)    # lo: full range
    return out


def segment_offsets(nseg: int = 65536, seed: int = 12, lo: int = 16, hi: int = 1 << 20) -> np.ndarray:
    """int64 offsets of nseg segments with lengths floor(exp(U(ln lo, ln hi)))."""
    rng = np.random.default_rng(seed)
    lens = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=nseg))).astype(np.int64)
    lens = np.clip(lens, lo, hi)
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def segmented_keys(offsets: np.ndarray, kt: int, seed: int) -> np.ndarray:
    n = int(offsets[-1])
    if kt == U32:
        return uniform_u32(n, seed)
    if kt == U64:
        return uniform_u64(n, seed)
    raise ValueError("segmented workloads use u32 or u64 keys")


# ---- counter-based keys (random access: any range of the stream can be produced on
# its own, on the host or on the GPU, with identical values) ------------------------

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def counter_u64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of SplitMix64 from initial state `seed`: output i
    is mix(seed + (i + 1) * 0x9E3779B97F4A7C15) (all arithmetic mod 2^64)."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def counter_u32(seed: int, start: int, count: int) -> np.ndarray:
    """High halves of counter_u64."""
    return (counter_u64(seed, start, count) >> np.uint64(32)).astype(np.uint32)


def _signed(c: int) -> int:
    return c - (1 << 64) if c >= 1 << 63 else c


def counter_torch(seed: int, start: int, count: int, bits: int, device) -> "torch.Tensor":
    """counter_u64 (bits 64, as int64) or counter_u32 (bits 32, as int32) computed on
    `device` with int64 arithmetic (wrapping multiplies; right shifts masked to be
    logical), in pieces of 2^26."""
    import torch
    out = torch.empty(count, dtype=torch.int64 if bits == 64 else torch.int32, device=device)
    piece = 1 << 26
    for p0 in range(0, count, piece):
        m = min(piece, count - p0)
        i = torch.arange(start + p0 + 1, start + p0 + m + 1, dtype=torch.int64, device=device)
        z = _signed(seed % (1 << 64)) + i * _signed(_GAMMA)
        z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _signed(_M1)
        z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _signed(_M2)
        z = z ^ ((z >> 31) & ((1 << 33) - 1))
        if bits == 64:
            out[p0:p0 + m] = z
        else:
            hi = (z >> 32) & 0xFFFFFFFF                 # the high half, in [0, 2^32)
            out[p0:p0 + m] = torch.where(hi >= (1 << 31), hi - (1 << 32), hi).to(torch.int32)
    return out


def lognormal_mixture_u64(n: int, seed: int = 15, ncomp: int = 8, dup_frac: float = 0.10,
                          dup_pool: int = 1 << 20, dup_s: float = 1.2) -> np.ndarray:
    """Mixture of ncomp lognormal components (weights 1/ncomp, mu ~ U[10, 40],
    sigma ~ U[0.1, 2]); key = floor(exp(mu + sigma z)), draws >= 2^64 redrawn.  A
    fraction dup_frac of the keys are duplicates taken from a pool of dup_pool
    mixture keys by Zipf(dup_s) rank; positions are shuffled."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(10.0, 40.0, size=ncomp)
    sigma = rng.uniform(0.1, 2.0, size=ncomp)

    def draw(m: int) -> np.ndarray:
        out = np.empty(m, dtype=np.uint64)
        filled = 0
        while filled < m:
            c = min(_CHUNK, m - filled)
            comp = rng.integers(0, ncomp, size=c)
            v = np.exp(mu[comp] + sigma[comp] * rng.standard_normal(c))
            v = v[v < 18446744073709549568.0]       # largest double below 2^64
            v = np.floor(v).astype(np.uint64)
            out[filled:filled + v.size] = v[:m - filled]
            filled += min(v.size, m - filled)
        return out

    ndup = int(round(dup_frac * n))
    base = draw(n - ndup)
    pool = draw(dup_pool)
    dups = pool[_zipf_ranks(rng, ndup, dup_pool, dup_s)]
    keys = np.concatenate([base, dups])
    rng.shuffle(keys)
    return keys


# ---- named configurations ---------------------------------------------------------

C2_DISTRIBUTIONS = ("uniform", "zipf", "8distinct", "sorted", "reverse", "almost", "m3killer")


def c2(dist: str, n: int) -> np.ndarray:
    return {
        "uniform": lambda: uniform_u64(n, 2),
        "zipf": lambda: zipf_u64(n, 3),
        "8distinct": lambda: few_distinct_u64(n, 4),
        "sorted": lambda: sorted_u64(n, 5),
        "reverse": lambda: reverse_u64(n, 5),
        "almost": lambda: almost_sorted_u64(n, 5, 6),
        "m3killer": lambda: median3_killer_u64(n - (n % 2)),
    }[dist]()


C3_CASES = {
    "f32_normal": (F32, lambda n: normal_f32(n, 7), 250_000_000),
    "f32_exponential": (F32, lambda n: exponential_f32(n, 8), 250_000_000),
    "f64_uniform": (F64, lambda n: uniform_f64(n, 9), 100_000_000),
    "u16_uniform": (U16, lambda n: uniform_u16(n, 10), 200_000_000),
    "u128": (U128, lambda n: u128_keys(n, 11), 50_000_000),
}
