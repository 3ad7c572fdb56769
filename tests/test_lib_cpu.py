"""CPU-side checks of the HIP library: it loads, and it exports every entry
point that include/tvlbm.h declares (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1004_5059_amd import tvlbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:tvlbm|tvnet)_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(tvlbm.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(tvlbm.LIB_PATH)
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            names += _declared(h)
    assert len(names) > 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_entry_points():
    if not os.path.exists(tvlbm.LIB_PATH):
        pytest.skip("library not built")
    assert tvlbm.tvlbm_strerror(tvlbm.TVLBM_ENONFINITE).startswith("non-finite")
    assert tvlbm.tvlbm_num_variants() >= 4


def test_descriptor_layout_matches_header():
    # offsets of the C struct with natural alignment on x86-64
    d = tvlbm.tvlbm_desc
    assert d.ld.offset == 24 and d.tau.offset == 32 and d.collide.offset == 48
    assert d.wall_lo_ux.offset == 64 and d.dy.offset == 96 and d.stream.offset == 120
    assert ctypes.sizeof(d) == 128


def test_stream_copy_rejects_bad_arguments():
    """The copy helper's checks run on the host before anything is enqueued:
    sizes that are not a multiple of 16 bytes, misaligned or null pointers."""
    if not os.path.exists(tvlbm.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(tvlbm.LIB_PATH)
    f = lib.tvlbm_stream_copy
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    a, b = 0x10000, 0x20000  # never dereferenced: every call below fails its checks
    assert f(a, b, 24, None) == tvlbm.TVLBM_EINVAL      # not a multiple of 16
    assert f(a + 4, b, 32, None) == tvlbm.TVLBM_EINVAL  # misaligned source
    assert f(a, b + 8, 32, None) == tvlbm.TVLBM_EINVAL  # misaligned destination
    assert f(None, b, 32, None) == tvlbm.TVLBM_EINVAL
    assert f(a, None, 32, None) == tvlbm.TVLBM_EINVAL
    assert f(a, b, -16, None) == tvlbm.TVLBM_EINVAL
    assert f(a, b, 0, None) == tvlbm.TVLBM_OK           # nothing to copy
