"""OpenMP versions of the paper's CPU kernels (Section 2: BFS-Conventional,
BFS-Hybrid dagger, BFS-VisitedBitmap), timed on the host's cores as a
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

KINDS = {"conventional": 0, "hybrid": 1, "visited_bitmap": 2}


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
            lib.omp_bfs.argtypes = [i64, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
            lib.omp_bfs.restype = i64
            _lib = lib
    return _lib


def bfs(g, source: int, kind: str = "visited_bitmap", threads: int = 0, want_parent: bool = True,
        alpha: int = 14, beta: int = 24):
    """Runs one search; returns (dist, parent or None, seconds, levels).
    `threads` = 0 uses OpenMP's default (OMP_NUM_THREADS or all cores)."""
    lib = load()
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    dist = np.empty(g.n, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32) if want_parent else None
    secs = ctypes.c_double()
    levels = lib.omp_bfs(g.n, rp.ctypes.data, col.ctypes.data, int(source), KINDS[kind], int(alpha), int(beta),
                         int(threads), dist.ctypes.data, parent.ctypes.data if want_parent else None,
                         ctypes.byref(secs))
    return dist, parent, secs.value, int(levels)


def max_threads() -> int:
    """Threads OpenMP uses by default here."""
    lib = ctypes.CDLL("libgomp.so.1")
    lib.omp_get_max_threads.restype = ctypes.c_int
    return int(lib.omp_get_max_threads())
