"""ctypes marshalling for libbfs.so (see include/bfs.h for the semantics)."""
from __future__ import annotations

import ctypes
import os
import sys
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libbfs.so")
_lock = threading.Lock()
_lib = None

BFS_OK = 0
BFS_ERR_INVALID_ARG = 1
BFS_ERR_OUT_OF_MEMORY = 2
BFS_ERR_DEVICE = 3
BFS_ERR_BUSY = 4
BFS_ERR_NOT_READY = 5
BFS_INPUT_DEVICE = 0x1
BFS_VALIDATE = 0x2
BFS_VALIDATE_SYMMETRY = 0x4
BFS_ROWPTR32 = 0x8
BFS_SORT_NEIGHBORS = 0x10

BFS_POLICY_AUTO = 0
BFS_POLICY_ALPHA_BETA = 1
BFS_POLICY_FRONTIER_5PCT = 2
BFS_POLICY_TD_ONLY = 3

BFS_LOOP_AUTO = 0
BFS_LOOP_HOST = 1
BFS_LOOP_GRAPH = 2
BFS_LOOP_PERSISTENT = 3
BFS_LOOP_QUEUED = 4
BFS_TD_VISITED_BITMAP = 0
BFS_TD_DIST_CAS = 1
BFS_TD_DIST_PLAIN = 2
BFS_TD_DIST_PLAIN_CULL = 3

BFS_REQ_QUEUED = 0
BFS_REQ_RUNNING = 1
BFS_REQ_DONE = 2
BFS_REQ_FAILED = 3

_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_vp, _f32, _f64 = ctypes.c_void_p, ctypes.c_float, ctypes.c_double


class bfs_params(ctypes.Structure):
    _fields_ = [(name, _i32) for name in (
        "policy", "alpha", "beta", "td_wave_degree", "td_block_degree", "bu_wave_degree",
        "block_size", "loop", "graph_chunk_levels", "collect_timing", "msbfs_block_size",
        "msbfs_bu_percent", "graph_td_blocks", "bu_blocks", "queue_ahead", "td_visited")]


class bfs_level_stats(ctypes.Structure):
    _fields_ = [("level", _i32), ("direction", _i32), ("frontier", _i64), ("frontier_edges", _i64),
                ("unvisited_edges", _i64), ("discovered", _i64), ("scanned", _i64),
                ("examined", _i64), ("ms", _f32), ("pad", _f32)]


class bfs_run_stats(ctypes.Structure):
    _fields_ = [("source", _i32), ("levels", _i32), ("reached", _i64), ("edges", _i64),
                ("device_ms", _f64), ("host_ms", _f64), ("loop", _i32), ("policy", _i32)]


class bfs_graph_info(ctypes.Structure):
    _fields_ = [("n", _i64), ("nnz", _i64), ("isolated", _i64), ("max_degree", _i64),
                ("device_bytes", _i64), ("row_ptr_bytes", _i32), ("device", _i32)]


class bfs_req_stats(ctypes.Structure):
    _fields_ = [("t_submit_ns", _i64), ("t_admit_ns", _i64), ("t_done_ns", _i64),
                ("levels", _i32), ("batch_lanes", _i32), ("edges", _i64)]


class BfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libbfs error {code}: {msg}")
        self.code = code


_SIGS = {
    "bfs_last_error": ([], ctypes.c_char_p),
    "bfs_default_params": ([_vp], ctypes.c_int),
    "bfs_create_graph": ([_i64, _i64, _vp, _vp, _u32, _vp], ctypes.c_int),
    "bfs_destroy_graph": ([_vp], ctypes.c_int),
    "bfs_graph_set_stream": ([_vp, _vp], ctypes.c_int),
    "bfs_graph_copy_csr": ([_vp, _vp, _vp], ctypes.c_int),
    "bfs_set_params": ([_vp, _vp], ctypes.c_int),
    "bfs_get_params": ([_vp, _vp], ctypes.c_int),
    "bfs_graph_info_get": ([_vp, _vp], ctypes.c_int),
    "bfs_run": ([_vp, _i32, _vp, _vp], ctypes.c_int),
    "bfs_get_run_stats": ([_vp, _vp, _vp, _i32], ctypes.c_int),
    "bfs_run_batch": ([_vp, _vp, _i32, _vp], ctypes.c_int),
    "bfs_run_batch_noalloc": ([_vp, _vp, _i32, _vp], ctypes.c_int),
    "bfs_serve_create": ([ctypes.c_size_t, _i32, _vp], ctypes.c_int),
    "bfs_serve_destroy": ([_vp], ctypes.c_int),
    "bfs_serve_submit": ([_vp, _vp, _i32, _vp, _vp, _vp], ctypes.c_int),
    "bfs_serve_poll": ([_vp, _u64, _vp, _vp], ctypes.c_int),
}


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libbfs.so.  Raises ImportError when it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise ImportError(f"{_LIB_PATH} is missing: build it with "
                                  "`python -m paper_2503_00430_amd.build`")
            try:  # share PyTorch's HIP runtime when it is available
                import torch  # noqa: F401
            except ImportError:
                pass
            lib = ctypes.CDLL(_LIB_PATH)
            for name, (args, res) in _SIGS.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = res
            _lib = lib
    return _lib


def bfs_last_error() -> str:
    return load_library().bfs_last_error().decode()


def _check(rc: int):
    if rc != BFS_OK:
        raise BfsError(rc, bfs_last_error())


def _dev_ptr(t, dtype, n, name):
    """Device pointer of a contiguous torch tensor with `n` elements."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor with {n} elements")
    return t.data_ptr()


class Graph:
    """Owner of a bfs_graph_t handle."""

    def __init__(self, handle, n: int, nnz: int):
        self.handle = handle
        self.n = n
        self.nnz = nnz

    def close(self):
        if self.handle:
            _check(load_library().bfs_destroy_graph(self.handle))
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # During interpreter shutdown the HIP runtime (and torch's use of it)
        # may already be torn down: a graph still open then is left to the
        # process exit instead of issuing frees, graph and stream destroys.
        # (The check is bound at definition: module globals such as `sys`
        # may already be cleared when this runs at shutdown.)
        if _finalizing():
            return
        try:
            if self.handle and _lib is not None:
                _lib.bfs_destroy_graph(self.handle)
                self.handle = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def bfs_create_graph(row_ptr, col_idx, flags: int = 0) -> Graph:
    """row_ptr int64[n+1], col_idx int32[nnz]: numpy arrays (host) or device
    tensors (then BFS_INPUT_DEVICE is added)."""
    lib = load_library()
    try:
        import torch
        is_dev = isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda
    except ImportError:
        is_dev = False
    if is_dev:
        n = row_ptr.numel() - 1
        nnz = col_idx.numel()
        rp = _dev_ptr(row_ptr, torch.int64, n + 1, "row_ptr")
        ci = _dev_ptr(col_idx, torch.int32, nnz, "col_idx") if nnz else None
        flags |= BFS_INPUT_DEVICE
        keep = (row_ptr, col_idx)
    else:
        rpa = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cia = np.ascontiguousarray(col_idx, dtype=np.int32)
        n, nnz = len(rpa) - 1, len(cia)
        rp, ci = rpa.ctypes.data, (cia.ctypes.data if nnz else None)
        keep = (rpa, cia)
    h = _vp()
    _check(lib.bfs_create_graph(n, nnz, rp, ci, flags, ctypes.byref(h)))
    del keep
    return Graph(h, n, nnz)


def bfs_destroy_graph(g: Graph):
    g.close()


def bfs_graph_copy_csr(g: Graph):
    """The device-resident CSR in its stored row order: (row_ptr int64[n+1],
    col_idx int32[nnz]) numpy arrays."""
    rp = np.empty(g.n + 1, np.int64)
    col = np.empty(max(g.nnz, 1), np.int32)
    _check(load_library().bfs_graph_copy_csr(g.handle, rp.ctypes.data, col.ctypes.data))
    return rp, col[:g.nnz]


def bfs_graph_set_stream(g: Graph, stream=None):
    """stream: torch.cuda.Stream, an integer hipStream_t, or None (null stream)."""
    s = getattr(stream, "cuda_stream", stream)
    _check(load_library().bfs_graph_set_stream(g.handle, _vp(s or 0)))


def bfs_default_params() -> dict:
    p = bfs_params()
    _check(load_library().bfs_default_params(ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in bfs_params._fields_ if f != "reserved"}


def bfs_get_params(g: Graph) -> dict:
    p = bfs_params()
    _check(load_library().bfs_get_params(g.handle, ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in bfs_params._fields_ if f != "reserved"}


def bfs_set_params(g: Graph, **changes):
    """Update named tunables (fields of bfs_params); others keep their value."""
    cur = bfs_get_params(g)
    unknown = set(changes) - set(cur)
    if unknown:
        raise KeyError(f"unknown parameters {sorted(unknown)}")
    cur.update(changes)
    p = bfs_params(**cur)
    _check(load_library().bfs_set_params(g.handle, ctypes.byref(p)))


def bfs_graph_info_get(g: Graph) -> dict:
    i = bfs_graph_info()
    _check(load_library().bfs_graph_info_get(g.handle, ctypes.byref(i)))
    return {f: getattr(i, f) for f, _ in bfs_graph_info._fields_}


def bfs_run(g: Graph, source: int, dist, parent=None):
    """dist: device int32 tensor [n]; parent: device int32 tensor [n] or None."""
    import torch
    d = _dev_ptr(dist, torch.int32, g.n, "dist")
    p = _dev_ptr(parent, torch.int32, g.n, "parent")
    _check(load_library().bfs_run(g.handle, int(source), d, p))


def bfs_get_run_stats(g: Graph, max_levels: int = 1 << 16):
    """Returns (run dict, list of per-level dicts) of the last bfs_run."""
    lib = load_library()
    st = bfs_run_stats()
    _check(lib.bfs_get_run_stats(g.handle, ctypes.byref(st), None, 0))
    n = max(0, min(st.levels, max_levels))
    lv = (bfs_level_stats * max(n, 1))()
    _check(lib.bfs_get_run_stats(g.handle, ctypes.byref(st), lv, n))
    run = {f: getattr(st, f) for f, _ in bfs_run_stats._fields_}
    levels = [{f: getattr(lv[i], f) for f, _ in bfs_level_stats._fields_ if f != "pad"}
              for i in range(n)]
    return run, levels


def bfs_run_batch(g: Graph, sources, dist8):
    """sources: host int32 array (k <= 64); dist8: device uint8 tensor [k, n]."""
    import torch
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = len(src)
    d = _dev_ptr(dist8, torch.uint8, k * g.n, "dist8")
    _check(load_library().bfs_run_batch(g.handle, src.ctypes.data, k, d))


def bfs_run_batch_noalloc(g: Graph, sources, dist8):
    """As bfs_run_batch, with the library's fixed scratch array (allocates
    nothing on the device)."""
    import torch
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = len(src)
    d = _dev_ptr(dist8, torch.uint8, k * g.n, "dist8")
    _check(load_library().bfs_run_batch_noalloc(g.handle, src.ctypes.data, k, d))


BFS_NOALLOC_SCRATCH_BYTES = 128 << 20


class Server:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self, _finalizing=sys.is_finalizing):
        # as Graph.__del__: nothing is issued once the interpreter is shutting down
        if _finalizing():
            return
        try:
            if self.handle and _lib is not None:
                _lib.bfs_serve_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def close(self):
        if self.handle:
            _check(load_library().bfs_serve_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def bfs_serve_create(hbm_budget_bytes: int, max_lanes: int = 64) -> Server:
    h = _vp()
    _check(load_library().bfs_serve_create(int(hbm_budget_bytes), int(max_lanes), ctypes.byref(h)))
    return Server(h)


def bfs_serve_destroy(s: Server):
    s.close()


def bfs_serve_submit(s: Server, g: Graph, source: int, dist, parent=None) -> int:
    import torch
    d = _dev_ptr(dist, torch.int32, g.n, "dist")
    p = _dev_ptr(parent, torch.int32, g.n, "parent")
    t = _u64()
    _check(load_library().bfs_serve_submit(s.handle, g.handle, int(source), d, p, ctypes.byref(t)))
    return int(t.value)


def bfs_serve_poll(s: Server, ticket: int):
    """Returns (state, stats dict)."""
    state = _i32()
    st = bfs_req_stats()
    _check(load_library().bfs_serve_poll(s.handle, int(ticket), ctypes.byref(state), ctypes.byref(st)))
    return int(state.value), {f: getattr(st, f) for f, _ in bfs_req_stats._fields_}
