"""The C-ABI library loads and exports every function include/gbgpu.h
declares (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbgpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbgpu_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    import paper_1805_05208_amd as gb
    if not os.path.exists(gb.LIB_PATH):
        from paper_1805_05208_amd import _build
        _build.build()
    return gb.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["gbgpu_load_csr", "gbgpu_bfs", "gbgpu_wbfs", "gbgpu_submit", "gbgpu_poll",
                     "gbgpu_bfs_multi", "gbgpu_bfs_batch", "gbgpu_last_error",
                     "gbgpu_bellman_ford", "gbgpu_widest_path", "gbgpu_bc",
                     "gbgpu_ldd", "gbgpu_connectivity", "gbgpu_compress", "gbgpu_decompress",
                     "gbgpu_bfs_compressed", "gbgpu_bfs_simple", "gbgpu_bfs_many"]:
        assert required in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_names_match_header(libpath):
    import paper_1805_05208_amd as gb
    assert sorted(gb.EXPORTED) == declared_functions()


def test_version_and_error_string(libpath):
    import paper_1805_05208_amd as gb
    L = gb.lib()
    assert L.gbgpu_version() >= 10000
    # a NULL graph is rejected before any device work
    st = L.gbgpu_graph_info(None, None, None, None)
    assert st == gb.E_INVALID
    assert b"NULL" in L.gbgpu_last_error()


def test_server_arena_allocator_selftest(libpath):
    """The server's first-fit arena (host logic) against a reference bitmap."""
    import paper_1805_05208_amd as gb
    L = gb.lib()
    for seed in range(1, 6):
        assert L.gbgpu_debug_arena_selftest(seed, 4000) == gb.OK, L.gbgpu_last_error()


def test_load_limits_refused_before_device_work(libpath):
    """Sizes beyond the library's limits are refused by argument checks that
    run before any device call (so this runs on the CPU): n >= 2^31 - 1 and
    m >= 2^31 give E_UNSUPPORTED, a missing SYMMETRIC flag or a NULL array
    E_INVALID.  The pointers passed are never dereferenced."""
    import paper_1805_05208_amd as gb
    L = gb.lib()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never read: the size checks come first
    assert L.gbgpu_load_csr(2**31 - 1, 10, fake, fake, None, gb.SYMMETRIC, None,
                            ctypes.byref(out)) == gb.E_UNSUPPORTED
    assert b"2^31" in L.gbgpu_last_error()
    assert L.gbgpu_load_csr(100, 2**31, fake, fake, None, gb.SYMMETRIC, None,
                            ctypes.byref(out)) == gb.E_UNSUPPORTED
    assert b"2^31 - 1" in L.gbgpu_last_error()
    assert L.gbgpu_load_csr(100, 10, fake, fake, None, 0, None,
                            ctypes.byref(out)) == gb.E_INVALID
    assert L.gbgpu_load_csr(100, 10, None, fake, None, gb.SYMMETRIC, None,
                            ctypes.byref(out)) == gb.E_INVALID
    assert L.gbgpu_load_csr(0, 0, fake, fake, None, gb.SYMMETRIC, None,
                            ctypes.byref(out)) == gb.E_INVALID
    assert out.value is None
