"""Invariant checker for BFS results (test infrastructure only).

Independent of both the serial oracle and the GPU library: it never runs a
search itself.  It checks the properties that characterise a correct BFS
distance array and BFS tree on an undirected graph, so it can judge results
at any size, including those whose parents legitimately differ from the
oracle's (Section 2: racing writers may record different discoverers).

Distance invariants (dist int32, -1 = unreached):
  D1  dist[s] == 0, and dist[v] >= -1 everywhere.
  D2  on every edge with both ends reached, |dist[u] - dist[v]| <= 1.
  D3  no edge joins a reached and an unreached vertex.
  D4  every reached v != s has a neighbour at dist[v] - 1.
  D5  the number of reached vertices equals the size of s's connected
      component (scipy's connected_components, an independent routine).
D1-D4 together force dist to be the exact shortest-path distance within s's
component, and D3 + D5 force -1 exactly outside it.

Parent invariants (parent int32, -1 = unreached):
  P1  parent[s] == s.
  P2  for reached v != s: parent[v] is a neighbour of v and
      dist[parent[v]] == dist[v] - 1.
  P3  parent[v] == -1 exactly when dist[v] == -1.
"""
from __future__ import annotations

import numpy as np


def _rows(row_ptr: np.ndarray) -> np.ndarray:
    n = len(row_ptr) - 1
    deg = np.diff(row_ptr)
    return np.repeat(np.arange(n, dtype=np.int32), deg)


def validate(g, source: int, dist: np.ndarray, parent: np.ndarray | None = None,
             check_component: bool = True) -> list[str]:
    """Return the list of violated invariants (empty when the result is valid)."""
    errs: list[str] = []
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col_idx)
    n = len(rp) - 1
    dist = np.asarray(dist)
    if dist.shape != (n,):
        return [f"dist has shape {dist.shape}, expected ({n},)"]
    if dist[source] != 0:
        errs.append(f"D1: dist[source={source}] = {dist[source]}")
    if (dist < -1).any():
        errs.append(f"D1: {(dist < -1).sum()} entries below -1")
    row = _rows(rp)
    du = dist[row]
    dv = dist[col]
    ru, rv = du >= 0, dv >= 0
    both = ru & rv
    bad = both & (np.abs(du.astype(np.int64) - dv) > 1)
    if bad.any():
        j = int(np.flatnonzero(bad)[0])
        errs.append(f"D2: {bad.sum()} edges with |d(u)-d(v)|>1, e.g. ({row[j]},{col[j]}) "
                    f"d={du[j]},{dv[j]}")
    cross = ru ^ rv
    if cross.any():
        j = int(np.flatnonzero(cross)[0])
        errs.append(f"D3: {cross.sum()} edges join reached and unreached, e.g. ({row[j]},{col[j]})")
    # D4: a neighbour one level closer.
    pred = both & (dv.astype(np.int64) == du.astype(np.int64) - 1)
    has_pred = np.zeros(n, dtype=bool)
    has_pred[row[pred]] = True
    need = (dist > 0)
    missing = need & ~has_pred
    if missing.any():
        v = int(np.flatnonzero(missing)[0])
        errs.append(f"D4: {missing.sum()} reached vertices lack a predecessor, e.g. v={v} d={dist[v]}")
    if check_component:
        from scipy.sparse import csr_matrix
        from scipy.sparse.csgraph import connected_components
        if col.size:
            a = csr_matrix((np.ones(len(col), np.int8), col.astype(np.int64), rp), shape=(n, n))
            _, lab = connected_components(a, directed=False)
            comp = int((lab == lab[source]).sum())
        else:
            comp = 1
        reached = int((dist >= 0).sum())
        if comp != reached:
            errs.append(f"D5: reached {reached} vertices, component of source has {comp}")
    if parent is not None:
        parent = np.asarray(parent)
        if parent.shape != (n,):
            return errs + [f"parent has shape {parent.shape}, expected ({n},)"]
        if parent[source] != source:
            errs.append(f"P1: parent[source] = {parent[source]}")
        unreached = dist < 0
        if (parent[unreached] != -1).any():
            errs.append(f"P3: {(parent[unreached] != -1).sum()} unreached vertices with a parent")
        other = (dist > 0)
        p = parent[other]
        if ((p < 0) | (p >= n)).any():
            errs.append(f"P2: {((p < 0) | (p >= n)).sum()} reached vertices with parent out of range")
        else:
            ok_level = dist[p].astype(np.int64) == dist[other].astype(np.int64) - 1
            if not ok_level.all():
                v = int(np.flatnonzero(other)[np.flatnonzero(~ok_level)[0]])
                errs.append(f"P2: {(~ok_level).sum()} parents not one level up, e.g. v={v}")
            # (parent[v], v) must be an edge: some CSR entry of row v equals parent[v].
            hit = col == parent[row]
            is_edge = np.zeros(n, dtype=bool)
            is_edge[row[hit]] = True
            miss = other & ~is_edge
            if miss.any():
                v = int(np.flatnonzero(miss)[0])
                errs.append(f"P2: {miss.sum()} parents are not neighbours, e.g. v={v} p={parent[v]}")
    return errs
