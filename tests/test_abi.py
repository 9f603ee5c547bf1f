"""The C ABI library loads and exports every symbol the header declares.

Host-only calls (sizing, argument checks that fail before any device work,
names, version) run without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apsp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apsp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2412_15122_amd import _native as N
    return N.load()


def test_header_declares_the_update_and_query_calls():
    names = declared_functions()
    for required in ("apsp_cold", "apsp_add_node", "apsp_remove_node", "apsp_update_edge", "apsp_query",
                     "apsp_query_nodes"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2412_15122_amd import _native as N
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, f"binding lacks {name}"


def test_constants_match_header(lib):
    from paper_2412_15122_amd import _native as N
    text = open(HEADER).read()
    assert int(re.search(r"#define APSP_INF (\d+)", text).group(1)) == N.APSP_INF == 1 << 30
    assert int(re.search(r"#define APSP_MAX_CAPACITY (\d+)", text).group(1)) == N.APSP_MAX_CAPACITY
    assert int(re.search(r"#define APSP_NOALLOC_MAX_CAPACITY (\d+)", text).group(1)) == N.APSP_NOALLOC_MAX_CAPACITY
    # the static working memory of the no-allocation edge update holds a graph
    # of the largest capacity it accepts, and stays modest
    P = N.APSP_NOALLOC_MAX_CAPACITY
    assert P * P // 8 + 1024 * P * 4 <= lib.apsp_noalloc_scratch_bytes() <= 32 << 20
    assert lib.apsp_abi_version() == int(re.search(r"#define APSP_ABI_VERSION (\d+)", text).group(1))
    for name in ("APSP_OK", "APSP_E_INVALID", "APSP_E_NOT_FOUND", "APSP_E_CAPACITY", "APSP_E_DEVICE", "APSP_E_VALUE"):
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert int(m.group(1)) == getattr(N, name)


def test_required_bytes(lib):
    from paper_2412_15122_amd import _native as N
    assert lib.apsp_required_bytes(0, 0) == 0
    assert lib.apsp_required_bytes(N.APSP_MAX_CAPACITY + 1, 0) == 0
    assert lib.apsp_required_bytes(10, 7) == 0    # minimax and widest together
    assert lib.apsp_required_bytes(10, 8) == 0    # an unknown bit
    assert lib.apsp_required_bytes(10, N.APSP_WIDEST | N.APSP_UNDIRECTED) == lib.apsp_required_bytes(10, 1)
    und = lib.apsp_required_bytes(16384, N.APSP_UNDIRECTED)
    dire = lib.apsp_required_bytes(16384, N.APSP_DIRECTED)
    mat = 16384 * 16384 * 4
    assert 2 * mat <= und < 2 * mat + (256 << 20)     # D + A + index + workspace
    assert dire - und >= mat                          # plus the transpose
    assert lib.apsp_required_bytes(100, 0) % 256 == 0


def test_cold_argument_checks_fail_before_device_work(lib):
    from paper_2412_15122_amd import _native as N
    h = ctypes.c_void_p()
    assert lib.apsp_cold(None, 4, 4, 0, 8, None, 0, None, None) == N.APSP_E_INVALID
    assert lib.apsp_cold(None, 4, 4, 0, 8, None, 0, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert b"adjacency" in lib.apsp_last_error()
    assert lib.apsp_cold(None, 0, 0, 3, 8, None, 0, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_cold(None, 9, 9, 0, 8, None, 0, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_cold(None, 0, 0, 0, 8, ctypes.c_void_p(256), 16, None, ctypes.byref(h)) == N.APSP_E_CAPACITY
    assert lib.apsp_cold(None, 0, 0, 0, 8, ctypes.c_void_p(257), 1 << 40, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert h.value is None


def test_null_handle_checks(lib):
    from paper_2412_15122_amd import _native as N
    assert lib.apsp_remove_node(None, 0) == N.APSP_E_INVALID
    assert lib.apsp_update_edge(None, 0, 1, 5) == N.APSP_E_INVALID
    assert lib.apsp_update_edge_noalloc(None, 0, 1, 5) == N.APSP_E_INVALID
    assert lib.apsp_add_node(None, None, None, None) == N.APSP_E_INVALID
    assert lib.apsp_graph_destroy(None) == N.APSP_OK


def test_kernel_names(lib):
    names = [lib.apsp_kernel_name(k).decode() for k in range(lib.apsp_kernel_count())]
    assert "mask_recompute" in names and "add_relax" in names and "fw_tiles" in names
    assert lib.apsp_kernel_name(-1) == b""


def test_batch_and_clone_host_checks(lib):
    from paper_2412_15122_amd import _native as N
    assert lib.apsp_batch_workspace_bytes(0, 1) == 0
    assert lib.apsp_batch_workspace_bytes(1, 0) == 0
    small = lib.apsp_batch_workspace_bytes(1, 1)
    big = lib.apsp_batch_workspace_bytes(512, 4096)
    assert small % 256 == 0 and big % 256 == 0 and big > small
    assert big < (48 << 20)                     # launch records and step tables only: graphs own their buffers
    h = ctypes.c_void_p()
    assert lib.apsp_batch_create(None, 1 << 20, 4, 4, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_batch_create(ctypes.c_void_p(257), 1 << 20, 4, 4, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_batch_create(ctypes.c_void_p(256), 16, 4, 4, ctypes.byref(h)) == N.APSP_E_CAPACITY
    assert lib.apsp_batch_create(ctypes.c_void_p(256), 1 << 20, 0, 4, ctypes.byref(h)) == N.APSP_E_INVALID
    assert h.value is None
    assert lib.apsp_batch_set_config(None, 0, 0, 0, 1) == N.APSP_E_INVALID
    assert lib.apsp_batch_run(None, None, 0, None, 0, None, None) == N.APSP_E_INVALID
    assert lib.apsp_batch_destroy(None) == N.APSP_OK
    assert lib.apsp_graph_clone(None, ctypes.c_void_p(256), 1 << 20, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_graph_clone(None, None, 0, None, None) == N.APSP_E_INVALID
    text = open(HEADER).read()
    assert int(re.search(r"#define APSP_BATCH_MAX_CAPACITY (\d+)", text).group(1)) == N.APSP_BATCH_MAX_CAPACITY
    for name in ("APSP_OP_ADD_NODE", "APSP_OP_REMOVE_NODE", "APSP_OP_UPDATE_EDGE", "APSP_OP_QUERY"):
        assert int(re.search(name + r"\s*=\s*(\d+)", text).group(1)) == getattr(N, name)
    assert ctypes.sizeof(N.BatchItem) == 48


def test_import_argument_checks_fail_before_device_work(lib):
    from paper_2412_15122_amd import _native as N
    h = ctypes.c_void_p()
    text = open(HEADER).read()
    for name in ("APSP_IMPORT_TRUSTED", "APSP_IMPORT_EXACT"):
        assert int(re.search(name + r"\s*=\s*(\d+)", text).group(1)) == getattr(N, name)
    fake = ctypes.c_void_p(256)
    # verify outside the two modes
    assert lib.apsp_import(fake, 4, fake, 4, 4, None, -1, 0, 8, fake, 1 << 30, None, 7, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    assert b"verify" in lib.apsp_last_error()
    # no matrix, or a leading dimension below n
    assert lib.apsp_import(fake, 4, None, 4, 4, None, -1, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    assert lib.apsp_import(fake, 4, fake, 3, 4, None, -1, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    # ids not strictly ascending, negative, or the largest int32 (its successor would overflow)
    for ids in ([0, 2, 2, 5], [-1, 0, 1, 2], [0, 1, 2, 2**31 - 1]):
        arr = (ctypes.c_int32 * 4)(*ids)
        assert lib.apsp_import(fake, 4, fake, 4, 4, arr, -1, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
            == N.APSP_E_INVALID
        assert b"ids" in lib.apsp_last_error()
    # the checks apsp_cold makes, with the import's name
    assert lib.apsp_import(fake, 4, fake, 4, 9, None, -1, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    assert lib.apsp_last_error().startswith(b"apsp_import")
    assert lib.apsp_import(fake, 4, fake, 4, 4, None, -1, 0, 8, fake, 16, None, 0, ctypes.byref(h)) \
        == N.APSP_E_CAPACITY
    assert lib.apsp_import(fake, 4, fake, 4, 4, None, -1, 0, 8, fake, 1 << 30, None, 0, None) == N.APSP_E_INVALID
    # next_id not above every id
    assert lib.apsp_import(fake, 4, fake, 4, 4, None, 3, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    assert b"next_id" in lib.apsp_last_error()
    assert lib.apsp_import(fake, 4, fake, 4, 4, None, -2, 0, 8, fake, 1 << 30, None, 0, ctypes.byref(h)) \
        == N.APSP_E_INVALID
    assert lib.apsp_next_id(None, None) == N.APSP_E_INVALID
    assert h.value is None


def test_grow_host_checks(lib):
    from paper_2412_15122_amd import _native as N
    h = ctypes.c_void_p()
    assert lib.apsp_grow(None, 8, ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) == N.APSP_E_INVALID
    assert lib.apsp_grow(None, 8, ctypes.c_void_p(256), 1 << 30, None, None) == N.APSP_E_INVALID
    assert h.value is None
