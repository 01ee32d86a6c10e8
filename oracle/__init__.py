"""The oracle: a plain, slow, obviously correct CPU model of what the GPU
library computes.  TEST INFRASTRUCTURE ONLY -- imported by the tests, the
smoke check and the benchmark's CPU-baseline leg, never by the library.

Contents
  bfs / bfs_timed          serial FIFO BFS in C (bfs_oracle.c); the paper's
                           problem statement (Section 1) and the common output
                           of Listings 1-3 (Section 2).
  level_stats              per-level frontier sizes and degree sums derived
                           from a distance array.
  replay_policy            the direction schedule that each switching rule of
                           Section 2 (BFS-Hybrid dagger: alpha/beta; BFS-Hybrid:
                           5 % of N) and the Section 3 graph classifier
                           (average degree < 7 => top-down only) produce on
                           those statistics.
  bottom_up_profile        vertices scanned / edges examined by a bottom-up
                           level with early exit (Section 2, BFS-Hybrid).
  algo_bytes               the byte model of each level.
  msbfs_dist8              batched distances saturated to uint8.
  validate                 independent invariant checker (validate.py).
  check_tree               the parent invariants of validate in one C pass
                           (for full-size trees whose distances are already
                           known to be exact).

All arithmetic here is exact integer arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from .validate import validate  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TD = 0
BU = 1

POLICY_ALPHA_BETA = "alpha_beta"
POLICY_FRONTIER_5PCT = "frontier_5pct"
POLICY_TD_ONLY = "td_only"
POLICY_AUTO = "auto"

DEFAULT_ALPHA = 14
DEFAULT_BETA = 24


def build(force: bool = False, mutant: int = 0, out: str | None = None) -> str:
    """Compile the C oracle (plain gcc).  `mutant` > 0 builds a deliberately
    wrong variant for the pin-strength tests; it is written to `out`."""
    target = out or _LIB
    if mutant == 0 and out is None and not force and os.path.exists(_LIB) \
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = target + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
           "-DORACLE_MUTANT=%d" % mutant, "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


def _bind(lib):
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_bfs.argtypes = [i64, vp, vp, i32, vp, vp, vp]
    lib.oracle_bfs.restype = i64
    lib.oracle_bottom_up_profile.argtypes = [i64, vp, vp, vp, i32, vp]
    lib.oracle_bottom_up_profile.restype = None
    lib.oracle_check_tree.argtypes = [i64, vp, vp, i32, vp, vp, vp]
    lib.oracle_check_tree.restype = None
    return lib


def load(path: str | None = None):
    """Load the oracle library (the default build, or a mutant at `path`)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _csr_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    return rp, col


def bfs_timed(g, source: int, want_parent: bool = True, lib=None):
    """Serial BFS from `source`.  Returns (dist, parent or None, seconds)."""
    lib = lib or load()
    rp, col = _csr_arrays(g)
    n = len(rp) - 1
    dist = np.empty(n, np.int32)
    parent = np.empty(n, np.int32) if want_parent else None
    secs = ctypes.c_double(0.0)
    r = lib.oracle_bfs(n, rp.ctypes.data, col.ctypes.data, int(source), dist.ctypes.data,
                       parent.ctypes.data if want_parent else None, ctypes.byref(secs))
    if r < 0:
        raise ValueError("oracle_bfs: bad arguments")
    return dist, parent, secs.value


def bfs(g, source: int, want_parent: bool = True, lib=None):
    """Serial BFS from `source`.  Returns (dist, parent or None)."""
    d, p, _ = bfs_timed(g, source, want_parent, lib)
    return d, p


def level_stats(g, dist: np.ndarray) -> dict:
    """Exact per-level quantities of a BFS result.

    h[L]   = |{v : dist[v] == L}|             (frontier expanded at level L)
    mf[L]  = sum of deg(v) over dist[v] == L   (edges leaving that frontier)
    mu[L]  = sum of deg(v) over v with dist[v] == -1 or dist[v] > L
             (edges of vertices still unvisited once level L-1 has finished,
             i.e. when the direction of level L is chosen)
    m_s    = (1/2) sum of deg(v) over reached v (undirected edges of the
             source's component: the TEPS edge count)
    """
    deg = np.diff(np.asarray(g.row_ptr, dtype=np.int64))
    reached = dist >= 0
    depth = int(dist.max()) + 1 if reached.any() else 0
    h = np.bincount(dist[reached], minlength=depth).astype(np.int64)
    mf = np.bincount(dist[reached], weights=deg[reached], minlength=depth).astype(np.int64)
    nnz = int(deg.sum())
    mu = nnz - np.cumsum(mf)  # after levels 0..L are visited
    # mu[L] as defined above = nnz - sum_{l <= L} mf[l]
    return {"n": int(len(dist)), "nnz": nnz, "depth": depth, "h": h, "mf": mf, "mu": mu,
            "m_s": int(deg[reached].sum()) // 2, "reached": int(reached.sum())}


def replay_policy(stats: dict, policy: str = POLICY_AUTO, alpha: int = DEFAULT_ALPHA,
                  beta: int = DEFAULT_BETA) -> list[int]:
    """Direction of every level (TD=0 / BU=1) that a switching rule takes.

    Level L expands frontier F_L (size h[L]); a run has `depth` = max dist + 1
    levels, the last of which finds nothing.  Level 0 is top-down (the paper's kernel
    starts with is_top_down = true).  The direction of level L+1 is chosen
    after level L from the new frontier:
      alpha_beta (Section 2, BFS-Hybrid dagger, after Beamer et al.):
        from TD go BU when m_f > m_u / alpha, i.e. m_f * alpha > m_u, where
        m_f = mf[L+1] and m_u = edges of still-unvisited vertices;
        from BU go back to TD when n_f < N / beta and n_f < n_f(previous),
        i.e. n_f * beta < N and h[L+1] < h[L]; otherwise keep the direction.
      frontier_5pct (Section 2, BFS-Hybrid): top-down while the new
        frontier is below 5 % of N, i.e. BU exactly when 20 * h[L+1] >= N.
      td_only: always TD.
      auto (Section 3 classifier): td_only when the average degree nnz / N
        is below 7, else alpha_beta.
    """
    n, nnz, depth = stats["n"], stats["nnz"], stats["depth"]
    h, mf, mu = stats["h"], stats["mf"], stats["mu"]
    if policy == POLICY_AUTO:
        policy = POLICY_TD_ONLY if nnz < 7 * n else POLICY_ALPHA_BETA
    dirs = [TD] if depth > 0 else []
    for L in range(depth - 1):  # choose the direction of level L+1 (F_{L+1} non-empty)
        n_new, mf_new, mu_new = int(h[L + 1]), int(mf[L + 1]), int(mu[L + 1])
        cur = dirs[-1]
        if policy == POLICY_TD_ONLY:
            nxt = TD
        elif policy == POLICY_FRONTIER_5PCT:
            nxt = BU if 20 * n_new >= n else TD
        elif policy == POLICY_ALPHA_BETA:
            if cur == TD:
                nxt = BU if mf_new * alpha > mu_new else TD
            else:
                nxt = TD if (n_new * beta < n and n_new < int(h[L])) else BU
        else:
            raise ValueError(policy)
        dirs.append(nxt)
    return dirs


def bottom_up_profile(g, dist: np.ndarray, level: int, lib=None) -> dict:
    """Scan work of a bottom-up level L (see bfs_oracle.c)."""
    lib = lib or load()
    rp, col = _csr_arrays(g)
    out = np.zeros(4, np.int64)
    d = np.ascontiguousarray(dist, dtype=np.int32)
    lib.oracle_bottom_up_profile(len(rp) - 1, rp.ctypes.data, col.ctypes.data, d.ctypes.data,
                                 int(level), out.ctypes.data)
    return {"unvisited": int(out[0]), "examined": int(out[1]), "found": int(out[2]),
            "full": int(out[3])}


def check_tree(g, source: int, dist: np.ndarray, parent: np.ndarray, lib=None) -> list[str]:
    """Parent invariants P1-P3 of validate.py (see there) checked in C, one
    pass over the rows; meant for distance arrays already shown exact.
    Returns the violated invariants (empty when the tree is valid)."""
    lib = lib or load()
    rp, col = _csr_arrays(g)
    n = len(rp) - 1
    d = np.ascontiguousarray(dist, dtype=np.int32)
    p = np.ascontiguousarray(parent, dtype=np.int32)
    if d.shape != (n,) or p.shape != (n,):
        return [f"dist/parent shapes {d.shape}/{p.shape}, expected ({n},)"]
    out = np.zeros(5, np.int64)
    lib.oracle_check_tree(n, rp.ctypes.data, col.ctypes.data, int(source), d.ctypes.data,
                          p.ctypes.data, out.ctypes.data)
    names = ["P1: parent[source] != source", "P3: parent set exactly where dist is not -1",
             "P2: parent one level up", "P2: parent is a neighbour"]
    return [f"{names[k]}: {int(out[k])} vertices violate it (first v={int(out[4])})"
            for k in range(4) if out[k]]


def bitmap_bytes(n: int) -> int:
    """Bytes of a bit-per-vertex map stored as 64-bit words."""
    return 8 * ((n + 63) // 64)


def algo_bytes(stats: dict, dirs: list[int], bu_profiles: dict, row_ptr_bytes: int,
               with_parent: bool) -> dict:
    """Bytes each level must move (the algorithmic byte model).

    W = row_ptr entry width, B = bitmap bytes (N bits), p = 4 if parents are
    written else 0, n_f = h[L], n_f' = h[L+1], m_f = mf[L]:
      init      : 4N + pN + B
      TD level  : 4 n_f (queue) + 2W n_f (row bounds) + 4 m_f (neighbour ids)
                  + B (visited bits) + (4 + p + 4 + 2W) n_f' (dist, parent,
                  queue append, row bounds of each new vertex for its degree)
      BU level  : B (visited) + W min(N+1, 2|U|) (row bounds) + 4 sum e_v
                  (neighbour ids up to the first hit) + B (frontier bits)
                  + 2B (next-frontier and visited words) + (4 + p) n_f'
    `bu_profiles[L]` is bottom_up_profile() of every BU level L.
    """
    n = stats["n"]
    h, mf = stats["h"], stats["mf"]
    B = bitmap_bytes(n)
    W = row_ptr_bytes
    p = 4 if with_parent else 0
    out = {"init": 4 * n + p * n + B, "levels": []}
    for L, d in enumerate(dirs):
        nf = int(h[L]) if L < len(h) else 0
        nf_new = int(h[L + 1]) if L + 1 < len(h) else 0
        if d == TD:
            b = 4 * nf + 2 * W * nf + 4 * int(mf[L] if L < len(mf) else 0) + B \
                + (4 + p + 4 + 2 * W) * nf_new
        else:
            prof = bu_profiles[L]
            b = B + W * min(n + 1, 2 * prof["unvisited"]) + 4 * prof["examined"] + B + 2 * B \
                + (4 + p) * nf_new
        out["levels"].append(int(b))
    return out


def msbfs_dist8(g, sources) -> np.ndarray:
    """Batched distances: row k holds min(dist from sources[k], 255), with
    255 also for unreached vertices; uint8 [k][N] row-major."""
    out = np.empty((len(sources), g.n), np.uint8)
    for k, s in enumerate(sources):
        d, _ = bfs(g, int(s), want_parent=False)
        out[k] = np.where((d < 0) | (d >= 255), 255, d).astype(np.uint8)
    return out
