"""OpenMP versions of the paper's CPU kernels (Section 2: BFS-Conventional,
BFS-NonAtomic, BFS-Hybrid with the 5 % rule, BFS-Hybrid dagger with the
alpha/beta rule, BFS-VisitedBitmap), timed on the host's cores as a
multicore context figure beside the GPU library and the serial oracle.

Neither the oracle nor part of the GPU library: the benchmark reports it
next to its serial-oracle CPU baseline, and CPU tests check its distances
against the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_omp.c")
_LIB = os.path.join(_HERE, "libbfs_omp.so")
_lock = threading.Lock()
_lib = None

# name: (top-down body, direction rule) of bfs_omp.c
#   body 0 compare-and-swap on dist, 1 plain test and store of dist
#   (duplicates allowed), 2 visited bitmap with atomic OR; rule 0 top-down
#   only, 1 the 5 % frontier rule, 2 alpha/beta
KINDS = {
    "conventional": (0, 0),            # BFS-Conventional
    "nonatomic": (1, 0),               # BFS-NonAtomic
    "hybrid": (1, 1),                  # BFS-Hybrid: NonAtomic top-down body, 5 % rule
    "hybrid_dagger": (1, 2),           # BFS-Hybrid dagger: alpha/beta rule
    "visited_bitmap": (2, 1),          # BFS-VisitedBitmap: bitmap on BFS-Hybrid
    "visited_bitmap_dagger": (2, 2),   # the bitmap with the alpha/beta rule
}


def build(force: bool = False) -> str:
    """Compile bfs_omp.c with gcc -fopenmp (generic x86-64 code, so the
    library runs on any host of this image)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            lib.omp_bfs.argtypes = [i64, vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp]
            lib.omp_bfs.restype = i64
            _lib = lib
    return _lib


def bfs(g, source: int, kind: str = "visited_bitmap", threads: int = 0, want_parent: bool = True,
        alpha: int = 14, beta: int = 24, return_entries: bool = False):
    """Runs one search; returns (dist, parent or None, seconds, levels), and
    with return_entries also the frontier entries over all levels
    (duplicates included).  `threads` = 0 uses OpenMP's default
    (OMP_NUM_THREADS or all cores)."""
    lib = load()
    body, rule = KINDS[kind]
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    dist = np.empty(g.n, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32) if want_parent else None
    secs = ctypes.c_double()
    entries = ctypes.c_int64()
    levels = lib.omp_bfs(g.n, rp.ctypes.data, col.ctypes.data, int(source), body, rule, int(alpha), int(beta),
                         int(threads), dist.ctypes.data, parent.ctypes.data if want_parent else None,
                         ctypes.byref(secs), ctypes.byref(entries))
    out = (dist, parent, secs.value, int(levels))
    return out + (int(entries.value),) if return_entries else out


def max_threads() -> int:
    """Threads OpenMP uses by default here."""
    lib = ctypes.CDLL("libgomp.so.1")
    lib.omp_get_max_threads.restype = ctypes.c_int
    return int(lib.omp_get_max_threads())
