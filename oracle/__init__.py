"""Scalar CPU oracle for the vectorized Quicksort (Blacher et al. 2022).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The GPU library never imports, links or calls it,
and it shares no code with the GPU library.

The arithmetic lives in plain C (vqs_oracle.c, one scalar routine per step of
the paper's method); this module only marshals numpy arrays through ctypes.
The learned-splitter model oracle is in oracle/mlp.py.

Key types use the interface numbering: 1 u16, 2 u32, 3 u64, 4 u128 (numpy
uint64 array of shape (n, 2): column 0 the low word, column 1 the high word),
5 f32, 6 f64, 7 i16, 8 i32, 9 i64, 10 k64v64 (a 64-bit key with 64-bit data as
a 128-bit key: column 1 the key, column 0 the data).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "vqs_oracle.c")
_CTX_SRC = os.path.join(_HERE, "context_sort.cpp")
_CTX_PATH = os.path.join(_HERE, "libcontext_sort.so")
_lock = threading.Lock()
_lib = None
_ctx = None

U16, U32, U64, U128, F32, F64 = 1, 2, 3, 4, 5, 6
I16, I32, I64, K64V64 = 7, 8, 9, 10
_DTYPES = {U16: np.uint16, U32: np.uint32, U64: np.uint64, U128: np.uint64,
           F32: np.float32, F64: np.float64, I16: np.int16, I32: np.int32, I64: np.int64,
           K64V64: np.uint64}
KEY_SIZE = {U16: 2, U32: 4, U64: 8, U128: 16, F32: 4, F64: 8, I16: 2, I32: 4, I64: 8, K64V64: 16}
PAIR_TYPES = (U128, K64V64)   # (n, 2) uint64 arrays: column 0 the low word, column 1 the high
NB_DEFAULT = 256


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "partitions", "keys_partitioned", "degenerate", "all_equal", "basecases",
        "heapsorts", "heapsort_keys", "max_depth", "depth_limit_used")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (strict IEEE: no FP contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC),
                                                  os.path.getmtime(os.path.join(_HERE, "oracle_body.h")),
                                                  os.path.getmtime(os.path.join(_HERE, "mlp_oracle.c"))):
            tmp = _LIB_PATH + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                                   "-fno-fast-math", "-Wall", "-Wno-unused-function",
                                   "-o", tmp, _SRC, os.path.join(_HERE, "mlp_oracle.c"), "-lm"])
            os.replace(tmp, _LIB_PATH)
        if force or not os.path.exists(_CTX_PATH) or os.path.getmtime(_CTX_PATH) < os.path.getmtime(_CTX_SRC):
            tmp = _CTX_PATH + ".tmp%d" % os.getpid()
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _CTX_SRC])
            os.replace(tmp, _CTX_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, vp, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        L.vqo_sort_segmented.argtypes = [vp, vp, u64, i32, i32, u64, u64, i64, ctypes.POINTER(Stats)]
        L.vqo_sort.argtypes = [vp, u64, i32, i32, u64, u64, i64, ctypes.POINTER(Stats)]
        L.vqo_choose_pivot.argtypes = [vp, u64, u64, i32, i32, u64, vp]
        L.vqo_choose_pivot_rng.argtypes = [vp, u64, u64, i32, i32, u64, i32, vp, vp]
        L.vqo_sort_segmented_rng.argtypes = [vp, vp, u64, i32, i32, u64, i32, vp, u64, i64, ctypes.POINTER(Stats)]
        L.vqo_sort_segmented_opts.argtypes = [vp, vp, u64, i32, i32, u64, i32, vp, u64, i64, i32,
                                              ctypes.POINTER(Stats)]
        L.vqo_partition_inplace.argtypes = [vp, u64, u64, i32, i32, vp]
        L.vqo_partition_inplace.restype = i64
        L.vqo_chacha20_block.argtypes = [vp, ctypes.c_uint32, vp, vp]
        L.vqo_chacha20_quarter_round.argtypes = [vp]
        L.vqo_pivot_offsets_rng.argtypes = [u64, i32, vp, u64, u64, u64, vp]
        L.vqo_partition.argtypes = [vp, u64, u64, i32, i32, vp]
        L.vqo_partition.restype = i64
        L.vqo_minmax.argtypes = [vp, u64, u64, i32, i32, vp, vp]
        L.vqo_basecase.argtypes = [vp, u64, i32, i32]
        L.vqo_heapsort.argtypes = [vp, u64, i32, i32]
        L.vqo_sfc64_raw.argtypes = [vp, vp, u64]
        L.vqo_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
        L.vqo_splitmix64_next.restype = u64
        L.vqo_seg_rng_state.argtypes = [u64, u64, u64, vp]
        L.vqo_multiply_shift.argtypes = [ctypes.c_uint32, u64]
        L.vqo_multiply_shift.restype = u64
        L.vqo_pivot_offsets.argtypes = [u64, u64, u64, u64, vp]
        L.vqo_default_depth_limit.argtypes = [u64]
        L.vqo_default_depth_limit.restype = u64
        L.vqo_green16.argtypes = [vp]
        L.vqo_merge_network.argtypes = [u64, vp]
        L.vqo_basecase_network.argtypes = [u64, vp, vp, vp]
        L.vqo_med3_u64.argtypes = [u64, u64, u64, i32]
        L.vqo_med3_u64.restype = u64
        L.vqo_key_size.argtypes = [i32]
        _mlp_signatures(L)
        _lib = L
    return _lib


def _mlp_signatures(L):
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    L.vqo_mlp_forward_f32.argtypes = [vp, vp, u64, vp]
    L.vqo_mlp_bucket_u64.argtypes = [vp, vp, u64, i32, vp]
    L.vqo_key_to_x_u64.argtypes = [vp, u64, vp]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_keys(keys: np.ndarray, kt: int) -> None:
    if not keys.flags.c_contiguous:
        raise ValueError("keys must be C-contiguous")
    if keys.dtype != _DTYPES[kt]:
        raise TypeError(f"key type {kt} needs dtype {_DTYPES[kt]}, got {keys.dtype}")
    if kt in PAIR_TYPES and (keys.ndim != 2 or keys.shape[1] != 2):
        raise ValueError("u128 / k64v64 keys are an (n, 2) uint64 array [lo, hi]")


def nkeys(keys: np.ndarray, kt: int) -> int:
    return keys.shape[0] if kt in PAIR_TYPES else keys.size


def _key_words(key):
    """A 256-bit ChaCha20 key as eight little-endian 32-bit words (or None)."""
    if key is None:
        return None
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(-1))
    if k.size != 8:
        raise ValueError("the ChaCha20 key is eight 32-bit words")
    return k


def sort(keys: np.ndarray, kt: int, ascending: bool = True, seed: int = 0,
         nb: int = NB_DEFAULT, depth_limit: int = -1, stats: bool = False, rng_key=None,
         inplace: bool = False):
    """Sort keys in place with the paper's method; returns stats if asked.  With
    rng_key (eight 32-bit words) the pivot sampler draws from ChaCha20 under that key
    (the secure generator option of Sec. 2.2) instead of SFC64 from the seed.  With
    inplace, Partition is the in-place bidirectional scan of Sec. 2.1 (64-key vectors,
    four per loop iteration) instead of the out-of-place split."""
    offs = np.array([0, nkeys(keys, kt) if keys.ndim else 0], dtype=np.int64)
    return sort_segmented(keys, offs, kt, ascending, seed, nb, depth_limit, stats, rng_key, inplace)


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, kt: int, ascending: bool = True,
                   seed: int = 0, nb: int = NB_DEFAULT, depth_limit: int = -1, stats: bool = False,
                   rng_key=None, inplace: bool = False):
    _check_keys(keys, kt)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    st = Stats()
    k = _key_words(rng_key)
    rc = lib().vqo_sort_segmented_opts(_ptr(keys), _ptr(offsets), offsets.size - 1, kt,
                                       int(bool(ascending)), seed, 1 if k is not None else 0,
                                       _ptr(k) if k is not None else None, nb, depth_limit,
                                       int(bool(inplace)), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError(f"vqo_sort_segmented failed: {rc}")
    return st.as_dict() if stats else None


def choose_pivot(keys: np.ndarray, b: int, e: int, kt: int, ascending: bool = True, seed: int = 0,
                 rng_key=None):
    _check_keys(keys, kt)
    out = np.zeros(2 if kt in PAIR_TYPES else 1, dtype=_DTYPES[kt])
    k = _key_words(rng_key)
    rc = lib().vqo_choose_pivot_rng(_ptr(keys), b, e, kt, int(bool(ascending)), seed, 1 if k is not None else 0,
                                    _ptr(k) if k is not None else None, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"vqo_choose_pivot failed: {rc}")
    return out if kt in PAIR_TYPES else out[0]


def partition(keys: np.ndarray, b: int, e: int, pivot, kt: int, ascending: bool = True) -> int:
    _check_keys(keys, kt)
    p = np.array(pivot, dtype=_DTYPES[kt]).reshape(-1)
    return int(lib().vqo_partition(_ptr(keys), b, e, kt, int(bool(ascending)), _ptr(p)))


def partition_inplace(keys: np.ndarray, b: int, e: int, pivot, kt: int, ascending: bool = True) -> int:
    """The in-place bidirectional Partition of Sec. 2.1 on [b, e); returns the bound."""
    _check_keys(keys, kt)
    p = np.array(pivot, dtype=_DTYPES[kt]).reshape(-1)
    return int(lib().vqo_partition_inplace(_ptr(keys), b, e, kt, int(bool(ascending)), _ptr(p)))


IP_LANES, IP_UNROLL = 64, 4          # the in-place Partition's vector and loop iteration
IP_BLOCK = IP_LANES * IP_UNROLL


def minmax(keys: np.ndarray, b: int, e: int, kt: int, ascending: bool = True):
    _check_keys(keys, kt)
    f = np.zeros(2 if kt in PAIR_TYPES else 1, dtype=_DTYPES[kt])
    l = np.zeros_like(f)
    if lib().vqo_minmax(_ptr(keys), b, e, kt, int(bool(ascending)), _ptr(f), _ptr(l)) != 0:
        raise ValueError("empty range")
    return (f, l) if kt in PAIR_TYPES else (f[0], l[0])


def plain_split_sizes(keys: np.ndarray, kt: int, levels: int = 8, seed: int = 0,
                      ascending: bool = True, nb: int = NB_DEFAULT, return_keys: bool = False):
    """Sizes of the ranges the paper's recursion (Alg. 1) holds after `levels` rounds of
    partitioning keys[0, n) (a copy): every range longer than the base-case size is
    split at ChoosePivot; a degenerate split repeats with the first key in sort order
    as pivot within the same round, and an all-equal range stays whole.  Ranges that
    stop splitting early keep their size.  Yardstick for a 2^levels-way splitter: these are
    the buckets plain pivot sampling makes."""
    a = np.ascontiguousarray(keys).copy()
    n = nkeys(a, kt)
    ranges = [(0, n)]
    for _ in range(levels):
        nxt = []
        for b, e in ranges:
            if e - b <= nb:
                nxt.append((b, e))
                continue
            bound = partition(a, b, e, choose_pivot(a, b, e, kt, ascending, seed), kt, ascending)
            if bound == e:
                first, last = minmax(a, b, e, kt, ascending)
                if np.array_equal(np.asarray(first), np.asarray(last)):
                    nxt.append((b, e))
                    continue
                bound = partition(a, b, e, first, kt, ascending)
            nxt += [(b, bound), (bound, e)]
        ranges = nxt
    sizes = np.array([e - b for b, e in ranges], dtype=np.int64)
    return (sizes, a) if return_keys else sizes


def basecase(keys: np.ndarray, kt: int, ascending: bool = True) -> None:
    _check_keys(keys, kt)
    if lib().vqo_basecase(_ptr(keys), nkeys(keys, kt), kt, int(bool(ascending))) != 0:
        raise ValueError("base case holds at most 1024 keys")


def heapsort(keys: np.ndarray, kt: int, ascending: bool = True) -> None:
    _check_keys(keys, kt)
    lib().vqo_heapsort(_ptr(keys), nkeys(keys, kt), kt, int(bool(ascending)))


def sfc64_raw(state, count: int) -> np.ndarray:
    st = np.array(state, dtype=np.uint64)
    out = np.zeros(count, dtype=np.uint64)
    lib().vqo_sfc64_raw(_ptr(st), _ptr(out), count)
    return out


def splitmix64(x: int, count: int):
    s = ctypes.c_uint64(x)
    return [int(lib().vqo_splitmix64_next(ctypes.byref(s))) for _ in range(count)]


def seg_rng_state(seed: int, b: int, e: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().vqo_seg_rng_state(seed, b, e, _ptr(out))
    return out


def multiply_shift(u: int, rng: int) -> int:
    return int(lib().vqo_multiply_shift(u, rng))


def pivot_offsets(seed: int, b: int, e: int, w: int, rng_key=None) -> np.ndarray:
    out = np.zeros(9, dtype=np.uint64)
    k = _key_words(rng_key)
    lib().vqo_pivot_offsets_rng(seed, 1 if k is not None else 0, _ptr(k) if k is not None else None, b, e, w,
                                _ptr(out))
    return out


def chacha20_block(key, counter: int, nonce) -> np.ndarray:
    """The ChaCha20 block function (RFC 8439 Sec. 2.3): sixteen 32-bit output words."""
    k = _key_words(key)
    nn = np.ascontiguousarray(np.asarray(nonce, dtype=np.uint32).reshape(3))
    out = np.zeros(16, dtype=np.uint32)
    lib().vqo_chacha20_block(_ptr(k), counter, _ptr(nn), _ptr(out))
    return out


def chacha20_quarter_round(a: int, b: int, c: int, d: int):
    v = np.array([a, b, c, d], dtype=np.uint32)
    lib().vqo_chacha20_quarter_round(_ptr(v))
    return tuple(int(x) for x in v)


def default_depth_limit(n: int) -> int:
    return int(lib().vqo_default_depth_limit(n))


def green16():
    out = np.zeros(120, dtype=np.uint32)
    n = lib().vqo_green16(_ptr(out))
    return [tuple(map(int, out[2 * i:2 * i + 2])) for i in range(n)]


def merge_network(length: int):
    out = np.zeros(length * 32, dtype=np.uint32)
    n = lib().vqo_merge_network(length, _ptr(out))
    return [tuple(map(int, out[2 * i:2 * i + 2])) for i in range(n)]


def basecase_network(n: int):
    """The module list BaseCase applies to n keys: (pairs as an (m, 2) array of cells,
    output order (the cell of the k-th key in sort order), cell count 16c)."""
    pairs = np.zeros(2 * 32768, dtype=np.uint32)
    order = np.zeros(1024, dtype=np.uint32)
    cells = np.zeros(1, dtype=np.uint32)
    m = lib().vqo_basecase_network(n, _ptr(pairs), _ptr(order), _ptr(cells))
    if m < 0:
        raise ValueError("BaseCase holds at most 1024 keys")
    c = int(cells[0])
    return pairs[:2 * m].reshape(m, 2).copy(), order[:c].copy(), c


def med3_u64(a: int, b: int, c: int, ascending: bool = True) -> int:
    return int(lib().vqo_med3_u64(a, b, c, int(bool(ascending))))


def parallel_sort(keys: np.ndarray, kt: int, threads: int, ascending: bool = True, seed: int = 0,
                  nb: int = NB_DEFAULT) -> None:
    """Sort keys in place with the oracle on `threads` host threads (timing only).

    The top levels of Alg. 1's recursion run as tasks: every range longer than
    n / (2 * threads) keys is split by ChoosePivot and Partition, the ranges of a
    level concurrently (a degenerate split leaves its range whole).  The remaining
    ranges are then sorted by the oracle's sort, handed to the threads longest first.
    The output is the sorted keys.  Below the top levels the recursion restarts per
    range (its pivots drawn for it as an array of its own, its depth limit from its
    length), so the recursion counters are not those of the one-threaded oracle."""
    import concurrent.futures as cf
    _check_keys(keys, kt)
    n = nkeys(keys, kt)
    ks = KEY_SIZE[kt]
    L = lib()
    asc = int(bool(ascending))
    big = max(n // (2 * max(threads, 1)), 64 // ks + 1, nb + 1)

    def split(r):
        b, e = r
        p = choose_pivot(keys, b, e, kt, ascending, seed)
        bound = partition(keys, b, e, p, kt, ascending)
        if bound in (b, e):
            return [(b, e, True)]
        return [(b, bound, False), (bound, e, False)]

    def leaf(r):
        b, e = r
        st = Stats()
        L.vqo_sort(_ptr(keys) + b * ks, e - b, kt, asc, seed, nb, -1, ctypes.byref(st))

    with cf.ThreadPoolExecutor(max_workers=max(threads, 1)) as ex:
        todo, leaves = [(0, n)], []
        while todo:
            nxt = []
            for parts in ex.map(split, todo):
                for b, e, whole in parts:
                    if whole or e - b <= big:
                        leaves.append((b, e))
                    else:
                        nxt.append((b, e))
            todo = nxt
        leaves.sort(key=lambda r: r[0] - r[1])
        list(ex.map(leaf, leaves))


def context_std_sort(keys: np.ndarray, kt: int, ascending: bool = True) -> None:
    """std::sort of the same keys (context timing next to the oracle; not a reference)."""
    global _ctx
    _check_keys(keys, kt)
    if _ctx is None:
        build()
        c = ctypes.CDLL(_CTX_PATH)
        c.ctx_std_sort.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        _ctx = c
    if _ctx.ctx_std_sort(_ptr(keys), nkeys(keys, kt), kt, int(bool(ascending))) != 0:
        raise ValueError("unknown key type")
