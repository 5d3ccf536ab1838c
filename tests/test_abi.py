"""The C-ABI library: it loads on a machine without a GPU and exports every entry
point include/vqs.h declares; argument checks that return before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vqs.h")
LIB = os.path.join(ROOT, "paper_2205_05982_amd", "libvqs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vqs_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2205_05982_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_interface():
    names = declared_functions()
    for n in ("vqs_sort", "vqs_sort_segmented", "vqs_sort_ex", "vqs_sort_segmented_ex",
              "vqs_get_stats", "vqs_strerror", "vqs_workspace_bytes"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_version(lib):
    lib.vqs_strerror.restype = ctypes.c_char_p
    assert lib.vqs_strerror(0) == b"success"
    assert lib.vqs_strerror(-2) == b"unknown key type"
    assert lib.vqs_version() >= 10000


def test_profile_modes(lib):
    """vqs_profile: 0 off, 1 every launch, 2 level partitions only; other values
    rejected (setting the mode touches no device)."""
    for mode in (1, 2, 0):
        assert lib.vqs_profile(mode) == 0
    assert lib.vqs_profile(3) == -1
    assert lib.vqs_profile(-1) == -1


def test_binding_profile_modes():
    """The binding passes the mode through and raises on a rejected one."""
    from paper_2205_05982_amd import vqs
    vqs.profile(2)
    vqs.profile(True)
    vqs.profile(False)
    with pytest.raises(vqs.VqsError):
        vqs.profile(7)


def test_argument_errors_return_before_any_device_call(lib):
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.vqs_sort_ex.argtypes = [vp, u64, i32, i32, vp, vp]
    assert lib.vqs_sort_ex(None, 10, 11, 1, None, None) == -2     # unknown key type
    assert lib.vqs_sort_ex(None, 10, 3, 2, None, None) == -1      # ascending not 0/1
    assert lib.vqs_sort_ex(None, 0, 3, 1, None, None) == 0        # nothing to sort
    assert lib.vqs_sort_ex(None, 10, 3, 1, None, None) == -1      # null keys
    assert lib.vqs_sort_ex(ctypes.c_void_p(0x1004), 10, 3, 1, None, None) == -1   # misaligned u64


def test_options_layout_matches_binding():
    from paper_2205_05982_amd import vqs
    # struct vqs_options: 2*u32, u64, i64, 2*u32, u64, 4*u32, 3*float, (pad) 2*u64, 3*u32 (+ pad),
    # u64, pointer, u64, 10*u32 (+ pad)
    assert ctypes.sizeof(vqs.Options) == 176
    assert vqs.Options.rng.offset == 128 and vqs.Options.rng_key.offset == 132
    assert vqs.Options.inplace.offset == 168
    assert vqs.Options.model_seed.offset == 72
    assert vqs.Options.train_steps.offset == 48
    assert vqs.Options.level_mode.offset == 88
    assert vqs.Options.total_keys.offset == 104
    assert vqs.Options.tile_variant.offset == 96
    assert vqs.Options.workspace_bytes.offset == 120
    assert ctypes.sizeof(vqs.Stats) == 20 * 8


def test_options_and_stats_layout_match_the_header(tmp_path):
    """The binding's structures against the C header itself, compiled with gcc."""
    import subprocess
    from paper_2205_05982_amd import vqs
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "vqs.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(vqs_options),'
        ' offsetof(vqs_options, train_steps), offsetof(vqs_options, model_seed),'
        ' offsetof(vqs_options, level_mode), sizeof(vqs_stats), offsetof(vqs_stats, train_loss),'
        ' offsetof(vqs_options, fallback_limit), offsetof(vqs_options, total_keys),'
        ' offsetof(vqs_options, workspace), offsetof(vqs_options, workspace_bytes),'
        ' offsetof(vqs_stats, bounded_global), offsetof(vqs_options, inplace)); return 0; }\n')
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(vqs.Options), vqs.Options.train_steps.offset, vqs.Options.model_seed.offset,
                   vqs.Options.level_mode.offset, ctypes.sizeof(vqs.Stats), vqs.Stats.train_loss.offset,
                   vqs.Options.fallback_limit.offset, vqs.Options.total_keys.offset,
                   vqs.Options.workspace.offset, vqs.Options.workspace_bytes.offset,
                   vqs.Stats.bounded_global.offset, vqs.Options.inplace.offset]


def test_noalloc_argument_errors_return_before_any_device_call(lib):
    """vqs_sort_noalloc checks its arguments before it touches a device."""
    from paper_2205_05982_amd import vqs
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.vqs_sort_noalloc.argtypes = [vp, u64, i32, i32, ctypes.POINTER(vqs.Options), vp]
    assert lib.vqs_sort_noalloc(None, 10, 11, 1, None, None) == -2     # unknown key type
    assert lib.vqs_sort_noalloc(None, 10, 3, 2, None, None) == -1      # ascending not 0/1
    assert lib.vqs_sort_noalloc(None, 0, 3, 1, None, None) == 0        # nothing to sort
    assert lib.vqs_sort_noalloc(None, 10, 3, 1, None, None) == -1      # null keys
    assert lib.vqs_sort_noalloc(ctypes.c_void_p(0x1004), 10, 3, 1, None, None) == -1   # misaligned u64
    learned = vqs.make_options(method=1)
    assert lib.vqs_sort_noalloc(ctypes.c_void_p(0x1000), 10, 3, 1, ctypes.byref(learned), None) == -1
    graph = vqs.make_options(use_graph=1)
    assert lib.vqs_sort_noalloc(ctypes.c_void_p(0x1000), 10, 3, 1, ctypes.byref(graph), None) == -1
    lib.vqs_strerror.restype = ctypes.c_char_p
    assert b"vqs_sort_noalloc" in lib.vqs_strerror(-7)


def test_stable_and_new_key_types_argument_errors(lib):
    """vqs_sort_stable rejects 128-bit key types and bad arguments before any device
    call; the signed and key+data types are known to every entry point."""
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.vqs_sort_stable.argtypes = [vp, u64, i32, i32, vp, vp, vp]
    assert lib.vqs_sort_stable(None, 10, 4, 1, None, None, None) == -2     # u128
    assert lib.vqs_sort_stable(None, 10, 10, 1, None, None, None) == -2    # k64v64
    assert lib.vqs_sort_stable(None, 10, 11, 1, None, None, None) == -2    # unknown
    assert lib.vqs_sort_stable(None, 10, 8, 2, None, None, None) == -1     # ascending not 0/1
    assert lib.vqs_sort_stable(None, 0, 8, 1, None, None, None) == 0
    assert lib.vqs_sort_stable(ctypes.c_void_p(0x1000), 10, 8, 1, ctypes.c_void_p(0x1004), None, None) == -1
    lib.vqs_sort_ex.argtypes = [vp, u64, i32, i32, vp, vp]
    for kt in (7, 8, 9, 10):
        assert lib.vqs_sort_ex(None, 10, kt, 1, None, None) == -1          # known type, null keys
    assert lib.vqs_sort_ex(ctypes.c_void_p(0x1008), 10, 10, 1, None, None) == -1   # k64v64 needs 16-byte alignment
    lib.vqs_workspace_bytes.restype = ctypes.c_uint64
    lib.vqs_workspace_bytes.argtypes = [u64, u64, i32, vp]
    assert lib.vqs_workspace_bytes(1000, 1, 9, None) == lib.vqs_workspace_bytes(1000, 1, 3, None)
    assert lib.vqs_workspace_bytes(1000, 1, 10, None) == lib.vqs_workspace_bytes(1000, 1, 4, None)
