"""The allocation-free entry point vqs_sort_noalloc, through the C interface: on two
calls in a row (the second with a smaller input, so the fixed scratch still holds the
first call's contents) its output and recursion counters equal those of vqs_sort_ex
on the same input, bit for bit; it rejects inputs too large for the fixed scratch
without touching them; and device memory in use does not change across its calls."""
import ctypes

import numpy as np
import pytest

from tests.helpers import F32, U16, U32, U64, U128, random_keys, to_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vqs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2205_05982_amd import vqs as v
    return v


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(vqs, t, n, kt, asc, **opts):
    o = vqs.make_options(**opts)
    return vqs.lib().vqs_sort_noalloc(ctypes.c_void_p(t.data_ptr()), n, kt, int(asc), ctypes.byref(o), _stream())


def _ex(vqs, t, n, kt, asc, **opts):
    o = vqs.make_options(**opts)
    return vqs.lib().vqs_sort_ex(ctypes.c_void_p(t.data_ptr()), n, kt, int(asc), ctypes.byref(o), _stream())


def _both(vqs, keys, kt, asc, **opts):
    """(noalloc output, its counters), (vqs_sort_ex output, its counters)."""
    import torch
    n = keys.shape[0]
    a, b = to_gpu(keys), to_gpu(keys)
    assert _noalloc(vqs, a, n, kt, asc, **opts) == 0
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    sa = vqs.get_stats()
    assert _ex(vqs, b, n, kt, asc, **opts) == 0
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    sb = vqs.get_stats()
    return (to_host(a), sa), (to_host(b), sb)


COUNTERS = ("partitions", "keys_partitioned", "degenerate", "all_equal", "basecases", "fallbacks",
            "fallback_keys", "max_depth", "levels", "solo_items")


@pytest.mark.parametrize("kt,asc,n1,n2", [
    (U64, True, 3_000_000, 200_000),      # several device-wide levels, then solo only
    (U32, True, 5_000_001, 1_000_003),    # look-back levels, ragged sizes
    (F32, False, 2_000_000, 77_777),
    (U128, True, 1_500_000, 40_000),
    (U16, False, 4_000_000, 300_000),     # many all-equal ranges
])
def test_two_calls_match_sort_ex(vqs, kt, asc, n1, n2):
    print(f"case: noalloc kt={kt} asc={asc} n1={n1} n2={n2}", flush=True)
    for i, n in enumerate((n1, n2)):
        keys = random_keys(kt, n, 100 + 10 * kt + i)
        (ga, sa), (gb, sb) = _both(vqs, keys, kt, asc)
        np.testing.assert_array_equal(ga, gb)
        assert {k: sa[k] for k in COUNTERS} == {k: sb[k] for k in COUNTERS}
        want = np.sort(keys, axis=0) if kt != U128 else keys[np.lexsort((keys[:, 0], keys[:, 1]))]
        if not asc:
            want = want[::-1]
        np.testing.assert_array_equal(ga, want)


def test_options_and_view_off_a_16_byte_boundary(vqs):
    """A view starting 8 bytes past a boundary and a forced depth limit (fallback mode)."""
    import torch
    print("case: noalloc unaligned view, depth_limit", flush=True)
    keys = random_keys(U64, 900_001, 7)
    base_a = to_gpu(np.concatenate([keys[:1], keys]))
    base_b = base_a.clone()
    a, b = base_a[1:], base_b[1:]
    n = keys.shape[0]
    assert _noalloc(vqs, a, n, U64, True, depth_limit=3, solo_max=8192) == 0
    torch.cuda.synchronize()
    assert vqs.last_error_bits() == 0
    sa = vqs.get_stats()
    assert _ex(vqs, b, n, U64, True, depth_limit=3, solo_max=8192) == 0
    torch.cuda.synchronize()
    sb = vqs.get_stats()
    assert sa["fallbacks"] > 0 and sa["fallbacks"] == sb["fallbacks"]
    np.testing.assert_array_equal(to_host(a), to_host(b))
    np.testing.assert_array_equal(to_host(a), np.sort(keys))


def test_rejects_what_does_not_fit(vqs):
    """Inputs beyond the fixed scratch return VQS_ESIZE and are left untouched; the
    learned method and hipGraph capture are rejected."""
    import torch
    print("case: noalloc size limit", flush=True)
    lib = vqs.lib()
    lib.vqs_workspace_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
    lib.vqs_workspace_bytes.restype = ctypes.c_uint64
    n = 1 << 20
    while lib.vqs_workspace_bytes(n, 1, U64, None) <= vqs.NOALLOC_SCRATCH_BYTES:
        n *= 2
    t = torch.arange(n, 0, -1, dtype=torch.int64, device="cuda")
    before = t.clone()
    assert _noalloc(vqs, t, n, U64, True) == -7
    torch.cuda.synchronize()
    assert torch.equal(t, before)
    small = to_gpu(random_keys(U64, 1000, 3))
    assert _noalloc(vqs, small, 1000, U64, True, method=1) == -1
    assert _noalloc(vqs, small, 1000, U64, True, use_graph=1) == -1
    assert _noalloc(vqs, small, 0, U64, True) == 0


def test_device_memory_unchanged_across_calls(vqs):
    """After a first call, further calls of either size leave free device memory as it
    was (the entry point allocates nothing)."""
    import torch
    print("case: noalloc memory", flush=True)
    keys1 = random_keys(U64, 2_000_000, 21)
    keys2 = random_keys(U64, 150_000, 22)
    a, b = to_gpu(keys1), to_gpu(keys2)
    a0, b0 = a.clone(), b.clone()
    assert _noalloc(vqs, a, a.numel(), U64, True) == 0
    torch.cuda.synchronize()
    a.copy_(a0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    assert _noalloc(vqs, a, a.numel(), U64, True) == 0
    assert _noalloc(vqs, b, b.numel(), U64, True) == 0
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0
    np.testing.assert_array_equal(to_host(a), np.sort(keys1))
    np.testing.assert_array_equal(to_host(b), np.sort(keys2))
    assert vqs.last_error_bits() == 0
