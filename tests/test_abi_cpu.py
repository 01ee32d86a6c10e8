"""CPU-only checks of the C interface: the library loads, exports every
function include/bfs.h declares, the Python binding mirrors those names, and
argument errors are reported without touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2503_00430_amd as bfs
    if not os.path.exists(bfs.library_path()):
        from paper_2503_00430_amd import build
        build.build()
    return bfs.load_library()


def test_header_declares_contract():
    names = _declared()
    for required in ("bfs_create_graph", "bfs_destroy_graph", "bfs_run", "bfs_run_batch",
                     "bfs_serve_create", "bfs_serve_submit", "bfs_serve_poll", "bfs_serve_destroy",
                     "bfs_last_error", "bfs_set_params", "bfs_get_run_stats"):
        assert required in names


def test_exports_every_declared_symbol(lib):
    import paper_2503_00430_amd as bfs
    out = subprocess.run(["nm", "-D", "--defined-only", bfs.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(lib, n)


def test_binding_mirrors_names(lib):
    import paper_2503_00430_amd as bfs
    for n in _declared():
        assert callable(getattr(bfs, n)), n


def test_struct_sizes_match_header(lib):
    from paper_2503_00430_amd import _lib as L
    # sizes fixed by the C layout in bfs.h
    assert ctypes.sizeof(L.bfs_params) == 16 * 4
    assert ctypes.sizeof(L.bfs_level_stats) == 2 * 4 + 6 * 8 + 2 * 4
    assert ctypes.sizeof(L.bfs_run_stats) == 4 + 4 + 8 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(L.bfs_req_stats) == 3 * 8 + 2 * 4 + 8


def test_argument_errors(lib):
    import paper_2503_00430_amd as bfs
    vp = ctypes.c_void_p
    h = vp()
    rp = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    assert lib.bfs_create_graph(2, 2, rp.ctypes.data, col.ctypes.data, 0, None) == 1
    assert lib.bfs_create_graph(0, 0, rp.ctypes.data, col.ctypes.data, 0, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph(1 << 31, 0, rp.ctypes.data, col.ctypes.data, 0, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph(2, -1, rp.ctypes.data, col.ctypes.data, 0, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph(2, 2, None, col.ctypes.data, 0, ctypes.byref(h)) == 1
    assert lib.bfs_create_graph(2, 2, rp.ctypes.data, col.ctypes.data, 0x100, ctypes.byref(h)) == 1
    assert "flags" in bfs.bfs_last_error()
    assert lib.bfs_destroy_graph(None) == 1
    assert lib.bfs_run(None, 0, None, None) == 1
    assert lib.bfs_run_batch(None, None, 1, None) == 1
    assert lib.bfs_set_params(None, None) == 1
    assert lib.bfs_get_run_stats(None, None, None, 0) == 1
    assert lib.bfs_graph_set_stream(None, None) == 1
    assert lib.bfs_serve_poll(None, 0, None, None) == 1
    assert lib.bfs_serve_submit(None, None, 0, None, None, None) == 1
    assert lib.bfs_serve_destroy(None) == 1
    assert lib.bfs_default_params(None) == 1


def test_default_params(lib):
    import paper_2503_00430_amd as bfs
    p = bfs.bfs_default_params()
    assert p["alpha"] == 14 and p["beta"] == 24 and p["policy"] == bfs.BFS_POLICY_AUTO
    assert p["block_size"] % 64 == 0
    assert p["td_wave_degree"] < p["td_block_degree"]


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_2503_00430_amd import _lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "_LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        L.load_library()


def test_loop_param_defaults(lib):
    """Defaults of the queued-loop lookahead and the bottom-up grid."""
    import paper_2503_00430_amd._lib as L
    d = L.bfs_default_params()
    assert d["queue_ahead"] == 2 and d["bu_blocks"] == 0 and d["td_visited"] == 0
