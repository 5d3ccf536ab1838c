"""Test helpers: moving numpy keys to and from the GPU and comparing stats."""
import numpy as np

U16, U32, U64, U128, F32, F64 = 1, 2, 3, 4, 5, 6

# Counters the oracle and the library keep in the same sense (oracle name, GPU name).
STAT_PAIRS = [("partitions", "partitions"), ("keys_partitioned", "keys_partitioned"),
              ("degenerate", "degenerate"), ("all_equal", "all_equal"), ("basecases", "basecases"),
              ("heapsorts", "fallbacks"), ("heapsort_keys", "fallback_keys"), ("max_depth", "max_depth")]


def to_gpu(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def assert_stats_equal(ost: dict, gst: dict):
    diffs = {o: (ost[o], gst[g]) for o, g in STAT_PAIRS if ost[o] != gst[g]}
    assert not diffs, f"oracle vs GPU recursion counters differ: {diffs}"


def random_keys(kt, n, seed):
    rng = np.random.default_rng(seed)
    if kt == U16:
        return rng.integers(0, 2**16, n, dtype=np.uint16)
    if kt == U32:
        return rng.integers(0, 2**32, n, dtype=np.uint32)
    if kt == U64:
        return rng.integers(0, 2**64, n, dtype=np.uint64)
    if kt == U128:
        k = np.empty((n, 2), np.uint64)
        k[:, 0] = rng.integers(0, 2**64, n, dtype=np.uint64)
        k[:, 1] = rng.integers(0, 4, n, dtype=np.uint64)
        return k
    if kt == F32:
        a = rng.standard_normal(n, dtype=np.float32) * 1e3
        a[a == 0] = 0.0
        return a
    a = rng.standard_normal(n) * 1e-3
    a[a == 0] = 0.0
    return a
