"""Python binding of libvqs.so (argument marshalling only).

Every step of the sort runs in the library's HIP kernels; PyTorch only provides
device memory and the current stream.  If the shared library is missing the
import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvqs.so")

U16, U32, U64, U128, F32, F64 = 1, 2, 3, 4, 5, 6
I16, I32, I64, K64V64 = 7, 8, 9, 10
PLAIN, LEARNED = 0, 1
KEY_SIZE = {U16: 2, U32: 4, U64: 8, U128: 16, F32: 4, F64: 8, I16: 2, I32: 4, I64: 8, K64V64: 16}

_DTYPE_TO_KT = {torch.float32: F32, torch.float64: F64, torch.int16: I16, torch.int32: I32,
                torch.int64: I64}
for _name, _kt in (("uint16", U16), ("uint32", U32), ("uint64", U64)):
    if hasattr(torch, _name):
        _DTYPE_TO_KT[getattr(torch, _name)] = _kt
_ERRORS = {-1: "invalid argument", -2: "unknown key type", -3: "workspace allocation failed",
           -4: "HIP runtime error", -5: "segment offsets decrease", -6: "device capacity check failed",
           -7: "input too large for the fixed scratch of vqs_sort_noalloc"}
NOALLOC_SCRATCH_BYTES = 256 << 20


class VqsError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERRORS.get(code, 'error')} ({code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("method", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("depth_limit", ctypes.c_int64),
                ("base_case", ctypes.c_uint32), ("local_keys", ctypes.c_uint32),
                ("solo_max", ctypes.c_uint64), ("use_graph", ctypes.c_uint32),
                ("validate", ctypes.c_uint32), ("train_steps", ctypes.c_uint32),
                ("batch", ctypes.c_uint32), ("sample_fraction", ctypes.c_float),
                ("overflow_factor", ctypes.c_float), ("learning_rate", ctypes.c_float),
                ("model_seed", ctypes.c_uint64), ("sample_seed", ctypes.c_uint64),
                ("level_mode", ctypes.c_uint32), ("fallback_limit", ctypes.c_uint32),
                ("tile_variant", ctypes.c_uint32), ("total_keys", ctypes.c_uint64),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("rng", ctypes.c_uint32), ("rng_key", ctypes.c_uint32 * 8),
                ("reserved0", ctypes.c_uint32), ("inplace", ctypes.c_uint32)]


FALLBACK_LIMIT_ZERO = 0xFFFFFFFF


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "partitions", "keys_partitioned", "degenerate", "all_equal", "basecases", "fallbacks",
        "fallback_keys", "max_depth", "levels", "level_tiles", "solo_items", "lds_partitions",
        "learned_buckets", "overflow_buckets", "max_bucket")] + [("train_loss", ctypes.c_double)] + [
        (n, ctypes.c_uint64) for n in ("hbm_read_keys", "hbm_write_keys", "bounded_lds", "bounded_global")]

    def as_dict(self):
        return {n: (float(getattr(self, n)) if n == "train_loss" else int(getattr(self, n)))
                for n, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("level", ctypes.c_int32), ("keys", ctypes.c_uint64),
                ("ms", ctypes.c_double)]


KERNEL_KINDS = {0: "clear", 1: "seed", 2: "level_partition", 3: "solo", 4: "learned_sample",
                5: "learned_train", 6: "learned_thresholds", 7: "learned_scatter", 8: "pivots"}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2205_05982_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        L.vqs_sort.argtypes = [vp, u64, i32, i32]
        L.vqs_sort_ex.argtypes = [vp, u64, i32, i32, ctypes.POINTER(Options), vp]
        L.vqs_sort_noalloc.argtypes = [vp, u64, i32, i32, ctypes.POINTER(Options), vp]
        L.vqs_sort_segmented.argtypes = [vp, vp, u64, i32, i32]
        L.vqs_sort_segmented_ex.argtypes = [vp, vp, u64, i32, i32, ctypes.POINTER(Options), vp]
        L.vqs_workspace_bytes.argtypes = [u64, u64, i32, ctypes.POINTER(Options)]
        L.vqs_workspace_bytes.restype = u64
        L.vqs_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.vqs_last_error_bits.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        L.vqs_strerror.argtypes = [i32]
        L.vqs_strerror.restype = ctypes.c_char_p
        L.vqs_profile.argtypes = [i32]
        L.vqs_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
        for name in ("vqs_profile", "vqs_profile_read", "vqs_sort", "vqs_sort_ex", "vqs_sort_noalloc",
                     "vqs_sort_segmented", "vqs_sort_segmented_ex",
                     "vqs_get_stats", "vqs_last_error_bits", "vqs_release", "vqs_version"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


RNG_SFC64, RNG_CHACHA20 = 0, 1


def make_options(**kw) -> Options:
    """vqs_options from keyword arguments; rng_key (eight 32-bit words) selects the
    ChaCha20 sampler unless rng says otherwise."""
    o = Options()
    o.struct_size = ctypes.sizeof(Options)
    for k, v in kw.items():
        if v is None:
            continue
        if k == "method" and isinstance(v, str):
            v = {"plain": PLAIN, "learned": LEARNED}[v]
        if k == "rng_key":
            words = [int(x) & 0xFFFFFFFF for x in v]
            if len(words) != 8:
                raise ValueError("rng_key is eight 32-bit words")
            o.rng_key = (ctypes.c_uint32 * 8)(*words)
            if "rng" not in kw:
                o.rng = RNG_CHACHA20
            continue
        setattr(o, k, v)
    return o


def key_type_of(t: torch.Tensor, key_type: int | None = None) -> int:
    if key_type is not None:
        return key_type
    if t.dim() == 2 and t.shape[1] == 2 and t.element_size() == 8:
        raise ValueError("pass key_type=U128, K64V64 (or U64, I64) explicitly for a 2-column tensor")
    kt = _DTYPE_TO_KT.get(t.dtype)
    if kt is None:
        raise TypeError(f"no key type for dtype {t.dtype}; pass key_type")
    return kt


def _nkeys(t: torch.Tensor, kt: int) -> int:
    return t.numel() * t.element_size() // KEY_SIZE[kt]


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("keys must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("keys must be contiguous")


def sort(t: torch.Tensor, ascending: bool = True, key_type: int | None = None, stream=None, **opts) -> torch.Tensor:
    """Sort t in place (the whole tensor is one array of keys); returns t."""
    _check(t)
    kt = key_type_of(t, key_type)
    o = make_options(**opts)
    rc = lib().vqs_sort_ex(ctypes.c_void_p(t.data_ptr()), _nkeys(t, kt), kt, int(bool(ascending)),
                           ctypes.byref(o), ctypes.c_void_p(_stream_handle(stream)))
    if rc != 0:
        raise VqsError(rc, "vqs_sort")
    return t


def sort_noalloc(t: torch.Tensor, ascending: bool = True, key_type: int | None = None, stream=None,
                 **opts) -> torch.Tensor:
    """Sort t in place with the allocation-free entry point (vqs_sort_noalloc): the
    plain method, every workspace buffer taken from the library's fixed per-device
    scratch of NOALLOC_SCRATCH_BYTES; raises VqsError(-7) for inputs that do not fit."""
    _check(t)
    kt = key_type_of(t, key_type)
    o = make_options(**opts)
    rc = lib().vqs_sort_noalloc(ctypes.c_void_p(t.data_ptr()), _nkeys(t, kt), kt, int(bool(ascending)),
                                ctypes.byref(o), ctypes.c_void_p(_stream_handle(stream)))
    if rc != 0:
        raise VqsError(rc, "vqs_sort_noalloc")
    return t


def sort_stable(t: torch.Tensor, ascending: bool = True, key_type: int | None = None, rows: bool = True,
                stream=None, **opts):
    """Stable sort of t in place (vqs_sort_stable); returns (t, rows) where rows[i] is
    the input position of the key now at i (int64 tensor), or (t, None)."""
    _check(t)
    kt = key_type_of(t, key_type)
    n = _nkeys(t, kt)
    r = torch.empty(n, dtype=torch.int64, device=t.device) if rows else None
    o = make_options(**opts)
    L = lib()
    L.vqs_sort_stable.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.POINTER(Options), ctypes.c_void_p]
    L.vqs_sort_stable.restype = ctypes.c_int
    rc = L.vqs_sort_stable(ctypes.c_void_p(t.data_ptr()), n, kt, int(bool(ascending)),
                           ctypes.c_void_p(r.data_ptr() if r is not None else 0), ctypes.byref(o),
                           ctypes.c_void_p(_stream_handle(stream)))
    if rc != 0:
        raise VqsError(rc, "vqs_sort_stable")
    return t, r


def sort_segmented(t: torch.Tensor, offsets: torch.Tensor, ascending: bool = True,
                   key_type: int | None = None, stream=None, **opts) -> torch.Tensor:
    """Sort every segment [offsets[i], offsets[i+1]) of t in place (offsets: int64 on the GPU)."""
    _check(t)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 GPU tensor")
    kt = key_type_of(t, key_type)
    o = make_options(**opts)
    rc = lib().vqs_sort_segmented_ex(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                     offsets.numel() - 1, kt, int(bool(ascending)), ctypes.byref(o),
                                     ctypes.c_void_p(_stream_handle(stream)))
    if rc != 0:
        raise VqsError(rc, "vqs_sort_segmented")
    return t


TUNED_FIELDS = ("solo_max", "local_keys", "base_case", "level_mode", "tile_variant")


def autotune_segmented(t: torch.Tensor, offsets: torch.Tensor, ascending: bool = True,
                       key_type: int | None = None, max_keys: int = 0, cache: str | None = None,
                       stream=None, **opts) -> dict:
    """Run the library's autotuner (vqs_autotune_segmented) on a copy of a prefix of
    the segments of t; returns {"solo_max", "local_keys", "base_case", "best_ms"}.

    With cache (a JSON file path), a result stored for the same key type, segment
    count, key count and device is returned without tuning, and a new result is
    stored there.  Pass the returned settings (minus best_ms) to sort_segmented."""
    import json
    _check(t)
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous int64 GPU tensor")
    kt = key_type_of(t, key_type)
    nseg = offsets.numel() - 1
    tag = f"{kt}:{int(bool(ascending))}:{nseg}:{_nkeys(t, kt)}:{max_keys}:{torch.cuda.get_device_name(t.device)}"
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
        if tag in store:
            return dict(store[tag])
    o = make_options(**opts)
    best = ctypes.c_float(0.0)
    L = lib()
    L.vqs_autotune_segmented.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(Options),
                                         ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]
    L.vqs_autotune_segmented.restype = ctypes.c_int
    rc = L.vqs_autotune_segmented(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), nseg, kt,
                                  int(bool(ascending)), max_keys, ctypes.byref(o), ctypes.byref(best),
                                  ctypes.c_void_p(_stream_handle(stream)))
    if rc != 0:
        raise VqsError(rc, "vqs_autotune_segmented")
    res = {k: int(getattr(o, k)) for k in TUNED_FIELDS}
    res["best_ms"] = float(best.value)
    if cache:
        store[tag] = res
        with open(cache, "w") as f:
            json.dump(store, f, indent=1)
    return res


def get_stats(stream=None) -> dict:
    st = Stats()
    rc = lib().vqs_get_stats(ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(st))
    if rc != 0:
        raise VqsError(rc, "vqs_get_stats")
    return st.as_dict()


def last_error_bits(stream=None) -> int:
    v = ctypes.c_uint32(0)
    rc = lib().vqs_last_error_bits(ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(v))
    if rc != 0:
        raise VqsError(rc, "vqs_last_error_bits")
    return int(v.value)


def workspace_bytes(n: int, key_type: int, nseg: int = 1, **opts) -> int:
    o = make_options(**opts)
    return int(lib().vqs_workspace_bytes(n, nseg, key_type, ctypes.byref(o)))


def release() -> None:
    lib().vqs_release()


def version() -> int:
    return int(lib().vqs_version())


def profile(enable) -> None:
    """Record HIP events around kernel launches of later calls: False/0 none, True/1
    every launch, 2 only the device-wide partition launches."""
    _rc(lib().vqs_profile(int(enable)), "vqs_profile")


def profile_read(stream=None, max_records: int = 4096) -> list:
    arr = (KernelTime * max_records)()
    cnt = ctypes.c_int(0)
    rc = lib().vqs_profile_read(ctypes.c_void_p(_stream_handle(stream)), arr, max_records, ctypes.byref(cnt))
    if rc != 0:
        raise VqsError(rc, "vqs_profile_read")
    return [{"kind": KERNEL_KINDS.get(arr[i].kind, str(arr[i].kind)), "level": arr[i].level,
             "keys": int(arr[i].keys), "ms": float(arr[i].ms)} for i in range(cnt.value)]


# ---- learned splitter pieces ----------------------------------------------------------

MLP_NBLOCK = 1155
MLP_NPARAM = 1153


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _sig():
    L = lib()
    vp, u64, u32, i32, f32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_float
    L.vqs_learned_fit.argtypes = [vp, u64, ctypes.POINTER(Options), vp, vp]
    L.vqs_mlp_forward.argtypes = [vp, vp, u64, vp, vp]
    L.vqs_mlp_gradient.argtypes = [vp, vp, vp, u32, vp, vp, vp]
    L.vqs_mlp_train.argtypes = [vp, vp, vp, vp, u64, u32, u32, f32, u64, i32, vp]
    L.vqs_mlp_init.argtypes = [vp, u64, vp, u64, vp]
    L.vqs_mlp_buckets.argtypes = [vp, vp, u64, vp, vp]
    L.vqs_learned_thresholds.argtypes = [vp, vp, vp, vp]
    L.vqs_learned_classify.argtypes = [vp, u64, vp, vp, vp, vp]
    for n in ("vqs_learned_fit", "vqs_mlp_forward", "vqs_mlp_gradient", "vqs_mlp_train", "vqs_mlp_init",
              "vqs_mlp_buckets", "vqs_learned_thresholds", "vqs_learned_classify"):
        getattr(L, n).restype = i32
    return L


def _rc(rc, what):
    if rc != 0:
        raise VqsError(rc, what)


def learned_fit(keys: torch.Tensor, stream=None, **opts) -> torch.Tensor:
    """Sample, sort the sample, compute targets and train; returns the 1155-float model."""
    _check(keys)
    params = torch.empty(MLP_NBLOCK, dtype=torch.float32, device=keys.device)
    o = make_options(**opts)
    _rc(_sig().vqs_learned_fit(_p(keys), keys.numel() * keys.element_size() // 8, ctypes.byref(o), _p(params),
                               ctypes.c_void_p(_stream_handle(stream))), "vqs_learned_fit")
    return params


def mlp_forward(params, x, stream=None):
    y = torch.empty_like(x)
    _rc(_sig().vqs_mlp_forward(_p(params), _p(x), x.numel(), _p(y), ctypes.c_void_p(_stream_handle(stream))),
        "vqs_mlp_forward")
    return y


def mlp_gradient(params, x, t, stream=None):
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _rc(_sig().vqs_mlp_gradient(_p(params), _p(x), _p(t), x.numel(), _p(g), _p(loss),
                                ctypes.c_void_p(_stream_handle(stream))), "vqs_mlp_gradient")
    return g, loss


def mlp_train(params, moments, x, t, steps, batch, lr, seed=17, sequential=False, stream=None):
    _rc(_sig().vqs_mlp_train(_p(params), _p(moments), _p(x), _p(t), x.numel(), steps, batch, lr, seed,
                             int(bool(sequential)), ctypes.c_void_p(_stream_handle(stream))), "vqs_mlp_train")


def mlp_init(params, seed, x, stream=None):
    _rc(_sig().vqs_mlp_init(_p(params), seed, _p(x), x.numel(), ctypes.c_void_p(_stream_handle(stream))),
        "vqs_mlp_init")


def mlp_buckets(params, keys, stream=None):
    out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    _rc(_sig().vqs_mlp_buckets(_p(params), _p(keys), keys.numel(), _p(out), ctypes.c_void_p(_stream_handle(stream))),
        "vqs_mlp_buckets")
    return out


def learned_thresholds(params, stream=None):
    thr = torch.empty(255, dtype=torch.int64, device=params.device)
    nvalid = torch.empty(1, dtype=torch.int32, device=params.device)
    _rc(_sig().vqs_learned_thresholds(_p(params), _p(thr), _p(nvalid), ctypes.c_void_p(_stream_handle(stream))),
        "vqs_learned_thresholds")
    return thr, nvalid


def learned_classify(keys, thr, nvalid, stream=None):
    out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    _rc(_sig().vqs_learned_classify(_p(keys), keys.numel(), _p(thr), _p(nvalid), _p(out),
                                    ctypes.c_void_p(_stream_handle(stream))), "vqs_learned_classify")
    return out
