"""Small named graphs with closed-form BFS distances, for tests.

Each builder returns (CSR, closed_form) where closed_form(s) gives the exact
distance array from source s, derived from the graph's structure alone.
"""
from __future__ import annotations

import numpy as np

import graphgen


def path(n):
    u = np.arange(n - 1); v = u + 1
    g = graphgen.from_edges(n, u, v, f"path{n}")
    return g, lambda s: np.abs(np.arange(n) - s)


def cycle(n):
    u = np.arange(n); v = (u + 1) % n
    g = graphgen.from_edges(n, u, v, f"cycle{n}")

    def f(s):
        d = np.abs(np.arange(n) - s)
        return np.minimum(d, n - d)
    return g, f


def star(n):
    u = np.zeros(n - 1, np.int64); v = np.arange(1, n)
    g = graphgen.from_edges(n, u, v, f"star{n}")

    def f(s):
        if s == 0:
            d = np.ones(n, np.int64); d[0] = 0
        else:
            d = np.full(n, 2, np.int64); d[0] = 1; d[s] = 0
        return d
    return g, f


def complete(n):
    iu, iv = np.triu_indices(n, 1)
    g = graphgen.from_edges(n, iu, iv, f"K{n}")

    def f(s):
        d = np.ones(n, np.int64); d[s] = 0
        return d
    return g, f


def complete_bipartite(a, b):
    u = np.repeat(np.arange(a), b); v = a + np.tile(np.arange(b), a)
    n = a + b
    g = graphgen.from_edges(n, u, v, f"K{a},{b}")

    def f(s):
        side = np.arange(n) < a
        d = np.where(side == side[s], 2, 1).astype(np.int64); d[s] = 0
        return d
    return g, f


def lattice(w, h):
    """w x h grid, id = r*w + c, 4-neighbour, no deletions."""
    ids = np.arange(w * h).reshape(h, w)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    g = graphgen.from_edges(w * h, u, v, f"lattice{w}x{h}")

    def f(s):
        r, c = divmod(np.arange(w * h), w)
        sr, sc = divmod(s, w)
        return np.abs(r - sr) + np.abs(c - sc)
    return g, f


def hypercube(k):
    n = 1 << k
    u = np.repeat(np.arange(n), k); v = u ^ (1 << np.tile(np.arange(k), n))
    g = graphgen.from_edges(n, u, v, f"Q{k}")

    def f(s):
        x = np.arange(n) ^ s
        return np.array([bin(int(t)).count("1") for t in x])
    return g, f


def binary_tree(n):
    """Complete binary tree in heap order: children of i are 2i+1, 2i+2."""
    v = np.arange(1, n); u = (v - 1) // 2
    g = graphgen.from_edges(n, u, v, f"bintree{n}")

    def f(s):
        assert s == 0
        return np.floor(np.log2(np.arange(n) + 1)).astype(np.int64)
    return g, f


def two_paths(n1, n2):
    """Disjoint union of two paths; vertices of the other path are unreached."""
    u = np.concatenate([np.arange(n1 - 1), n1 + np.arange(n2 - 1)])
    v = u + 1
    n = n1 + n2
    g = graphgen.from_edges(n, u, v, f"P{n1}+P{n2}")

    def f(s):
        x = np.arange(n)
        same = (x < n1) == (s < n1)
        return np.where(same, np.abs(x - s), -1)
    return g, f


def broom(k, t):
    """Hub 0 joined to leaves 1..k; leaf 1 continues into a path of t
    vertices (ids k+1..k+t)."""
    u = list(np.zeros(k, np.int64)) + [1] + list(range(k + 1, k + t))
    v = list(range(1, k + 1)) + [k + 1] + list(range(k + 2, k + t + 1))
    return graphgen.from_edges(k + t + 1, u, v, f"broom{k},{t}")


def random_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, m); v = rng.integers(0, n, m)
    return graphgen.from_edges(n, u, v, f"rand{n},{m},{seed}")


CLOSED_FORMS = {
    "path": lambda: path(37),
    "cycle_odd": lambda: cycle(31),
    "cycle_even": lambda: cycle(40),
    "star": lambda: star(50),
    "complete": lambda: complete(20),
    "bipartite": lambda: complete_bipartite(7, 11),
    "lattice": lambda: lattice(13, 9),
    "hypercube": lambda: hypercube(7),
    "binary_tree": lambda: binary_tree(100),
    "two_paths": lambda: two_paths(15, 9),
}


def deferred_rows(n=8192, nf=1000, seed=3):
    """Source 0 joined to the nf highest ids F; every other vertex gets one
    random neighbour in F (its largest id, so last in its sorted row) and
    0-4 random neighbours below F, so most rows have three non-frontier
    neighbours ahead of the frontier one.  Distances: 1 on F, 2 elsewhere."""
    rng = np.random.default_rng(seed)
    lo = n - nf
    us, vs = [np.zeros(nf, np.int64)], [np.arange(lo, n)]
    others = np.arange(1, lo)
    us.append(others); vs.append(rng.integers(lo, n, len(others)))
    k = rng.integers(0, 5, len(others))
    src = np.repeat(others, k)
    us.append(src); vs.append(rng.integers(1, lo, len(src)))
    u, v = np.concatenate(us), np.concatenate(vs)
    keep = u != v
    g = graphgen.from_edges(n, u[keep], v[keep], f"deferred{n}")

    def f(s):
        assert s == 0
        d = np.full(n, 2, np.int64); d[lo:] = 1; d[0] = 0
        return d
    return g, f


def summary_skip(seed=11):
    """A top-down level whose expected frontier is large but whose actual one
    is small, followed by a bottom-up level (alpha 75, beta 24).  Source 0 is
    joined to vertex 1 of a 40-clique in word 0; every clique vertex has two
    pendants, each alone in one of words 1..80, and every pendant thirty
    leaves (words 81..118); the upper half is a dense part the source cannot
    reach, so almost every edge end is unvisited.  Level 2 expands the clique
    (1 661 edges, about 1 640 expected finds against 4 per bitmap word =
    1 024) and finds 138; level 3, bottom-up, has a 138-vertex frontier (at
    most 2 per word = 512): a summary missing the pendants' bits would hide
    every leaf's frontier neighbour.  Distances: 0, 1 (vertex 1), 2 (the
    clique and vertex 1's pendants), 3 (the other pendants and vertex 1's
    pendants' leaves), 4 (the other leaves), unreached elsewhere."""
    n = 16384
    rng = np.random.default_rng(seed)
    core = np.arange(1, 41)
    pend = 64 * (1 + np.arange(80))
    leaves = 64 * 81 + np.arange(80 * 30)
    dense = np.arange(8192, n)
    m = len(dense) * 9
    a, b = np.triu_indices(40, 1)
    u = np.concatenate([[0], core[a], np.repeat(core, 2), np.repeat(pend, 30), rng.choice(dense, m)])
    v = np.concatenate([[1], core[b], pend, leaves, rng.choice(dense, m)])
    keep = u != v
    return graphgen.from_edges(n, u[keep], v[keep], "summary_skip")

