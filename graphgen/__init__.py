"""Seeded synthetic graph inputs (CSR) shared by the checker and the GPU path.

This module creates inputs only; it contains no breadth-first-search
arithmetic.  The graph families follow the shapes the paper evaluates
(Section 3, Table 1): R-MAT power-law graphs for the Kronecker /
small-diameter class, uniform random graphs for urand, and a perturbed 2D
lattice for the large-diameter road/mesh class.

All arrays are returned as numpy views of memory owned by the native
generator; the `CSR` object keeps that memory alive.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lock = threading.Lock()
_lib = None

# Fixed seeds of the synthetic workloads (one place, so that every consumer
# draws the same graphs and sources).
RMAT_SEED = 1000
RMAT_PERM_SEED = 2000
GRID_SEED = 3000
URAND_SEED = 4000
SOURCE_SEED = 5000


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with g++/OpenMP (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
               "-std=c++17", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            vp, i64, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
            lib.gg_free.argtypes = [vp]
            lib.gg_n.argtypes = [vp]; lib.gg_n.restype = i64
            lib.gg_nnz.argtypes = [vp]; lib.gg_nnz.restype = i64
            lib.gg_row_ptr.argtypes = [vp]; lib.gg_row_ptr.restype = ctypes.POINTER(i64)
            lib.gg_col.argtypes = [vp]; lib.gg_col.restype = ctypes.POINTER(i32)
            lib.gg_draw.argtypes = [u64, u64]; lib.gg_draw.restype = u64
            lib.gg_from_edges.argtypes = [i64, i64, vp, vp]; lib.gg_from_edges.restype = vp
            lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, u64, u64]; lib.gg_rmat.restype = vp
            lib.gg_urand.argtypes = [i64, ctypes.c_int, u64]; lib.gg_urand.restype = vp
            lib.gg_grid.argtypes = [i64, dbl, dbl, ctypes.c_int, u64]; lib.gg_grid.restype = vp
            lib.gg_sources.argtypes = [i64, vp, i64, u64, vp]; lib.gg_sources.restype = i64
            _lib = lib
    return _lib


class CSR:
    """Symmetric CSR graph: row_ptr int64[n+1], col_idx int32[nnz]."""

    def __init__(self, handle=None, name: str = "", seed: int = 0, row_ptr=None, col_idx=None):
        self._handle = handle
        self.name = name
        self.seed = seed
        if handle is not None:
            lib = _load()
            self.n = int(lib.gg_n(handle))
            self.nnz = int(lib.gg_nnz(handle))
            self.row_ptr = np.ctypeslib.as_array(lib.gg_row_ptr(handle), shape=(self.n + 1,))
            self.col_idx = (np.ctypeslib.as_array(lib.gg_col(handle), shape=(self.nnz,))
                            if self.nnz else np.zeros(0, np.int32))
        else:
            self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
            self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
            self.n = len(self.row_ptr) - 1
            self.nnz = int(self.row_ptr[-1])

    def __del__(self):
        h, self._handle = getattr(self, "_handle", None), None
        if h is not None and _lib is not None:
            _lib.gg_free(h)

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def __repr__(self):
        return f"CSR({self.name!r}, n={self.n}, nnz={self.nnz})"


def _wrap(h, name, seed):
    if not h:
        raise MemoryError(f"graph generator failed for {name}")
    return CSR(h, name=name, seed=seed)


def draw(seed: int, ctr: int) -> int:
    """Element `ctr` of the SplitMix64 sequence started at state `seed`."""
    return int(_load().gg_draw(seed & (2**64 - 1), ctr & (2**64 - 1)))


def from_edges(n: int, u, v, name: str = "edges") -> CSR:
    """Symmetric, deduplicated, self-loop-free CSR from endpoint pairs."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    assert u.shape == v.shape
    h = _load().gg_from_edges(n, len(u), u.ctypes.data, v.ctypes.data)
    return _wrap(h, name, 0)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int | None = None, perm_seed: int | None = None) -> CSR:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale samples."""
    seed = RMAT_SEED + scale if seed is None else seed
    perm_seed = RMAT_PERM_SEED + scale if perm_seed is None else perm_seed
    h = _load().gg_rmat(scale, edge_factor, a, b, c, seed, perm_seed)
    return _wrap(h, f"rmat{scale}_ef{edge_factor}", seed)


def urand(n: int, avg_degree: int, seed: int | None = None) -> CSR:
    """Uniform random graph with n * avg_degree / 2 sampled pairs."""
    seed = URAND_SEED + avg_degree if seed is None else seed
    h = _load().gg_urand(n, avg_degree, seed)
    return _wrap(h, f"urand{n}_d{avg_degree}", seed)


def grid(width: int, p_delete: float = 0.1, p_shortcut: float = 0.01, radius: int = 8,
         seed: int | None = None) -> CSR:
    """width x width lattice with edge deletion and short random shortcuts."""
    seed = GRID_SEED + int(width).bit_length() - 1 if seed is None else seed
    h = _load().gg_grid(width, p_delete, p_shortcut, radius, seed)
    return _wrap(h, f"grid{width}", seed)


def sources(g: CSR, k: int, seed: int | None = None) -> np.ndarray:
    """k distinct vertices drawn uniformly among those with degree > 0."""
    seed = SOURCE_SEED + g.seed if seed is None else seed
    out = np.empty(k, dtype=np.int32)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    got = _load().gg_sources(g.n, rp.ctypes.data, k, seed, out.ctypes.data)
    return out[:got].copy()
