"""The C-ABI library loads and exports every entry point that include/bfsc.h
declares; host-only arithmetic agrees with the oracle (no GPU needed)."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfsc.h")
LIB = os.path.join(ROOT, "paper_1704_00513_amd", "libbfsc.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfsc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1704_00513_amd import build
        build.build()
    from paper_1704_00513_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "bfsc_encode" in names and "bfsc_decode" in names and "bfsc_bfs_level" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1704_00513_amd import _lib
    assert set(declared()) <= set(_lib.exported_symbols())


def test_encode_bound_matches_oracle_bound_and_holds(lib):
    lib.bfsc_encode_bound.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]
    lib.bfsc_encode_bound.restype = ctypes.c_int
    for n, r in [(0, 1), (1, 1), (127, 3), (128, 1), (5000, 16), (10 ** 7, 1024)]:
        out = ctypes.c_size_t()
        assert lib.bfsc_encode_bound(n, r, ctypes.byref(out)) == 0
        assert out.value == oracle.encode_bound(n, r)


def test_status_strings_and_host_errors(lib):
    lib.bfsc_status_string.restype = ctypes.c_char_p
    assert lib.bfsc_status_string(3) == b"corrupt compressed stream"
    from paper_1704_00513_amd import _lib
    h = ctypes.c_void_p()
    assert lib.bfsc_create(None, 0, None) == 1          # NULL out -> INVAL
    assert lib.bfsc_create(ctypes.byref(h), -1, None) == 1
    lib.bfsc_mlp_param_count.restype = ctypes.c_int
    assert lib.bfsc_mlp_param_count() == 7011


def test_exchange_owner_limit_is_checked_on_the_host(lib):
    """The owners' candidate bitmaps are indexed by 32-bit word numbers:
    nseg * ceil(V/32) must not pass 2^32 - 1 - 2^16, and nseg * nseg segments
    form one batch (nseg <= 65535); at scale 26 that is 2047 owners.  The BFS
    and exchange workspaces need no GPU."""
    from paper_1704_00513_amd import _lib
    csr = _lib.CSR()
    csr.n_vertices = 1 << 26
    csr.n_arcs = 1 << 30
    out = ctypes.c_size_t()
    size = lib.bfsc_exchange_workspace_size
    for R in (63, 64, 256, 1024, 2047):
        assert size(ctypes.byref(csr), R, ctypes.byref(out)) == 0, R
    # R candidate bitmaps + the merge bitmap, V/8 bytes each at least
    assert out.value >= 2048 * (1 << 26) // 8
    assert size(ctypes.byref(csr), 2048, ctypes.byref(out)) == 1
    assert size(ctypes.byref(csr), 0, ctypes.byref(out)) == 1
    words = (1 << 32) - 1 - (1 << 16)
    csr.n_vertices = 32 * (words // 4096)
    assert size(ctypes.byref(csr), 4096, ctypes.byref(out)) == 0
    csr.n_vertices += 32
    assert size(ctypes.byref(csr), 4096, ctypes.byref(out)) == 1
    csr.n_vertices = 1024
    assert size(ctypes.byref(csr), 65535, ctypes.byref(out)) == 0
    assert size(ctypes.byref(csr), 65536, ctypes.byref(out)) == 1
    csr.n_vertices = (1 << 26) - 32
    bfs = ctypes.c_size_t()
    assert lib.bfsc_bfs_workspace_size(ctypes.byref(csr), ctypes.byref(bfs)) == 0
    assert bfs.value >= 3 * ((1 << 26) - 32) // 8  # visited, next-level and frontier bitmaps


def test_config_defaults_and_range_checks(lib):
    """bfsc_config: the defaults, and settings out of range refused on the
    host before any device is touched."""
    from paper_1704_00513_amd import _lib
    c = _lib.default_config()
    assert (c.selector, c.raw_below, c.resolve_literal, c.autotune, c.tune_cache) == (1, 32, 0, 0, None)
    assert c.raw_below == _lib.RAW_BELOW == oracle.RAW_BELOW
    h = ctypes.c_void_p()
    for field, bad in (("selector", 3), ("selector", -1), ("raw_below", 2049), ("resolve_literal", 2),
                       ("autotune", 5)):
        c = _lib.default_config()
        setattr(c, field, bad)
        assert lib.bfsc_create(ctypes.byref(h), 0, ctypes.byref(c)) == 1, field
    c = _lib.default_config()
    c.tune_cache = b"x" * 2000  # longer than the context keeps
    assert lib.bfsc_create(ctypes.byref(h), 0, ctypes.byref(c)) == 1
