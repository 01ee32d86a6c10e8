"""Pins of the oracle against facts that do not come from the oracle itself.

* closed forms of named graphs (path, cycle, star, complete, complete
  bipartite, lattice = Manhattan distance, hypercube = Hamming distance,
  complete binary tree = floor(log2(i+1)), disjoint union = unreached);
* library routines (scipy.sparse.csgraph, networkx) on random graphs;
* brute-force relaxation to a fixpoint on small graphs;
* the hand-worked fixture in tests/golden/;
* the independent invariant checker (validate.py), and that it rejects
  corrupted results;
* metamorphic relations (relabelling, symmetry of distance);
* deliberately wrong oracle builds (mutants) must each fail some pin.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", sorted(graphs.CLOSED_FORMS))
def test_closed_forms(name):
    g, f = graphs.CLOSED_FORMS[name]()
    srcs = [0] if name == "binary_tree" else sorted({0, g.n // 3, g.n - 1})
    for s in srcs:
        d, p = oracle.bfs(g, s)
        np.testing.assert_array_equal(d, f(s), err_msg=f"{name} s={s}")
        assert oracle.validate(g, s, d, p) == []


def test_petersen():
    # Petersen graph: outer 5-cycle, inner pentagram, spokes; every vertex has
    # 3 neighbours at distance 1 and the other 6 vertices at distance 2.
    u = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 0, 1, 2, 3, 4]
    v = [1, 2, 3, 4, 0, 7, 8, 9, 5, 6, 5, 6, 7, 8, 9]
    g = graphgen.from_edges(10, u, v)
    for s in range(10):
        d, _ = oracle.bfs(g, s)
        assert sorted(d.tolist()) == [0, 1, 1, 1, 2, 2, 2, 2, 2, 2]


def _scipy_dist(g, s):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    a = csr_matrix((np.ones(g.nnz), g.col_idx.astype(np.int64), g.row_ptr), shape=(g.n, g.n))
    d = shortest_path(a, unweighted=True, directed=False, indices=s)
    return np.where(np.isinf(d), -1, d).astype(np.int64)


@pytest.mark.parametrize("n,m,seed", [(50, 40, 1), (300, 900, 2), (2000, 3000, 3), (20000, 60000, 4)])
def test_vs_scipy(n, m, seed):
    g = graphs.random_graph(n, m, seed)
    for s in [0, n // 2, n - 1]:
        d, p = oracle.bfs(g, s)
        np.testing.assert_array_equal(d, _scipy_dist(g, s))
        assert oracle.validate(g, s, d, p) == []


def test_vs_networkx():
    nx = pytest.importorskip("networkx")
    g = graphs.random_graph(3000, 5000, 7)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    G.add_edges_from(zip(rows.tolist(), g.col_idx.tolist()))
    for s in [1, 99, 2999]:
        ref = np.full(g.n, -1)
        for k, v in nx.single_source_shortest_path_length(G, s).items():
            ref[k] = v
        d, _ = oracle.bfs(g, s)
        np.testing.assert_array_equal(d, ref)


def _brute_force(g, s):
    """Relax d[v] = min(d[v], d[u] + 1) over every edge until nothing changes."""
    inf = 10 ** 9
    d = [inf] * g.n
    d[s] = 0
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr)).tolist()
    cols = g.col_idx.tolist()
    changed = True
    while changed:
        changed = False
        for u, v in zip(rows, cols):
            if d[u] + 1 < d[v]:
                d[v] = d[u] + 1
                changed = True
    return np.array([x if x < inf else -1 for x in d])


@pytest.mark.parametrize("seed", range(6))
def test_vs_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 200))
    m = int(rng.integers(0, 3 * n))
    g = graphs.random_graph(n, m, seed)
    for s in {0, n - 1, n // 2}:
        d, _ = oracle.bfs(g, s)
        np.testing.assert_array_equal(d, _brute_force(g, s))


def test_handworked_fixture():
    fx = json.load(open(os.path.join(GOLDEN, "handworked_12v.json")))
    e = np.array(fx["edges"])
    g = graphgen.from_edges(fx["n"], e[:, 0], e[:, 1])
    d, p = oracle.bfs(g, fx["source"])
    np.testing.assert_array_equal(d, fx["dist"])
    assert oracle.validate(g, fx["source"], d, p) == []
    st = oracle.level_stats(g, d)
    assert st["h"].tolist() == fx["h"]
    assert st["mf"].tolist() == fx["mf"]
    assert st["mu"].tolist() == fx["mu"]
    assert st["m_s"] == fx["m_s"]


def test_isolated_source_and_single_vertex():
    g = graphgen.from_edges(5, [1, 2], [2, 3])  # 0 and 4 isolated
    d, p = oracle.bfs(g, 0)
    assert d.tolist() == [0, -1, -1, -1, -1] and p.tolist() == [0, -1, -1, -1, -1]
    g1 = graphgen.from_edges(1, [], [])
    d, p = oracle.bfs(g1, 0)
    assert d.tolist() == [0] and p.tolist() == [0]


def test_rejects_bad_source():
    g, _ = graphs.path(5)
    with pytest.raises(ValueError):
        oracle.bfs(g, 5)
    with pytest.raises(ValueError):
        oracle.bfs(g, -1)


def test_metamorphic_relabel_and_symmetry():
    g = graphs.random_graph(500, 1500, 11)
    rng = np.random.default_rng(5)
    perm = rng.permutation(g.n)  # new id of old vertex i is perm[i]
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    h = graphgen.from_edges(g.n, perm[rows], perm[g.col_idx])
    for s in [0, 17, 333]:
        d, _ = oracle.bfs(g, s)
        d2, _ = oracle.bfs(h, int(perm[s]))
        np.testing.assert_array_equal(d2[perm], d)
    # d(s,t) == d(t,s)
    D = np.stack([oracle.bfs(g, s)[0] for s in range(0, 500, 25)])
    for i, s in enumerate(range(0, 500, 25)):
        for j, t in enumerate(range(0, 500, 25)):
            assert D[i, t] == D[j, s]


def test_validator_rejects_corruptions():
    g = graphs.random_graph(400, 1200, 21)
    s = 3
    d, p = oracle.bfs(g, s)
    assert oracle.validate(g, s, d, p) == []
    reached = np.flatnonzero(d > 0)
    v = int(reached[len(reached) // 2])
    for delta in (+1, -1):
        d2 = d.copy(); d2[v] += delta
        assert oracle.validate(g, s, d2, None) != []
    d3 = d.copy(); d3[s] = 1
    assert oracle.validate(g, s, d3, None) != []
    d4 = d.copy(); d4[v] = -1
    assert oracle.validate(g, s, d4, None) != []
    p2 = p.copy(); p2[v] = v
    assert oracle.validate(g, s, d, p2) != []
    p3 = p.copy(); p3[v] = int(np.flatnonzero(d == d[v])[0])  # same level, not a valid parent
    if p3[v] != p[v]:
        assert oracle.validate(g, s, d, p3) != []
    p4 = p.copy(); p4[s] = -1
    assert oracle.validate(g, s, d, p4) != []
    # a vertex two levels up that is not adjacent
    far = np.flatnonzero(d == max(d[v] - 2, 0))
    p5 = p.copy(); p5[v] = int(far[0])
    assert oracle.validate(g, s, d, p5) != []


def test_msbfs_saturation():
    g, f = graphs.path(300)
    out = oracle.msbfs_dist8(g, [0, 299, 150])
    assert out.dtype == np.uint8 and out.shape == (3, 300)
    exp0 = np.minimum(f(0), 255)
    np.testing.assert_array_equal(out[0], exp0)
    assert out[0, 255] == 255 and out[0, 254] == 254
    np.testing.assert_array_equal(out[2], np.minimum(f(150), 255))
    g2, _ = graphs.two_paths(4, 3)
    out2 = oracle.msbfs_dist8(g2, [0])
    assert out2[0].tolist() == [0, 1, 2, 3, 255, 255, 255]


def _pin_failures(lib):
    """Run the pin suite against an oracle library; return failing pin names."""
    failed = []
    for name, mk in graphs.CLOSED_FORMS.items():
        g, f = mk()
        srcs = [0] if name == "binary_tree" else sorted({0, g.n // 3, g.n - 1})
        for s in srcs:
            d, p = oracle.bfs(g, s, lib=lib)
            if not np.array_equal(d, f(s)) or oracle.validate(g, s, d, p) != []:
                failed.append(f"{name}/{s}")
    g = graphs.random_graph(300, 900, 2)
    d, p = oracle.bfs(g, 0, lib=lib)
    if not np.array_equal(d, _scipy_dist(g, 0)) or oracle.validate(g, 0, d, p):
        failed.append("scipy")
    return failed


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6])
def test_mutants_are_caught(mutant, tmp_path):
    path = oracle.build(mutant=mutant, out=str(tmp_path / f"liboracle_m{mutant}.so"))
    lib = oracle.load(path)
    assert _pin_failures(lib), f"mutant {mutant} passed every pin"


def test_unmutated_passes_pins():
    assert _pin_failures(oracle.load()) == []


def test_check_tree_pins():
    """check_tree (C) accepts valid BFS trees and names each planted fault:
    a hand-built tree on a path, trees of the closed-form graphs, and the
    corruptions the Python validator is pinned with."""
    g, _ = graphs.path(6)
    d = np.array([2, 1, 0, 1, 2, 3], np.int32)
    assert oracle.check_tree(g, 2, d, np.array([1, 2, 2, 2, 3, 4], np.int32)) == []
    assert oracle.check_tree(g, 2, d, np.array([1, 2, 1, 2, 3, 4], np.int32))[0].startswith("P1")
    assert oracle.check_tree(g, 2, d, np.array([2, 2, 2, 2, 3, 4], np.int32))[0].startswith("P2: parent one")
    # vertex 3 is one level above vertex 0 but not its neighbour
    assert oracle.check_tree(g, 2, d, np.array([3, 2, 2, 2, 3, 4], np.int32))[0].startswith("P2: parent is a")
    g2, _ = graphs.two_paths(4, 3)
    d2, p2 = oracle.bfs(g2, 0)
    assert oracle.check_tree(g2, 0, d2, p2) == []
    p2b = p2.copy(); p2b[5] = 4
    assert oracle.check_tree(g2, 0, d2, p2b)[0].startswith("P3")
    p2c = p2.copy(); p2c[2] = -1
    assert oracle.check_tree(g2, 0, d2, p2c)[0].startswith("P3")
    for name, mk in graphs.CLOSED_FORMS.items():
        gc, _ = mk()
        dc, pc = oracle.bfs(gc, 0)
        assert oracle.check_tree(gc, 0, dc, pc) == [], name
    g = graphs.random_graph(400, 1200, 21)
    s = 3
    d, p = oracle.bfs(g, s)
    assert oracle.check_tree(g, s, d, p) == []
    v = int(np.flatnonzero(d > 0)[len(np.flatnonzero(d > 0)) // 2])
    p_self = p.copy(); p_self[v] = v
    assert oracle.check_tree(g, s, d, p_self) != []
    same = int(np.flatnonzero(d == d[v])[0])
    if same != p[v]:
        p_same = p.copy(); p_same[v] = same
        assert oracle.check_tree(g, s, d, p_same) != []
    # one level up but not adjacent: only the row scan can catch it
    up = [int(u) for u in np.flatnonzero(d == d[v] - 1)
          if u not in set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())]
    if up:
        p_far = p.copy(); p_far[v] = up[0]
        errs = oracle.check_tree(g, s, d, p_far)
        assert len(errs) == 1 and errs[0].startswith("P2: parent is a neighbour"), errs
    p_out = p.copy(); p_out[v] = g.n
    assert oracle.check_tree(g, s, d, p_out) != []
    # agrees with the Python validator on random valid and corrupted trees
    rng = np.random.default_rng(5)
    for _ in range(20):
        q = p.copy()
        w = int(rng.integers(g.n))
        q[w] = int(rng.integers(-1, g.n))
        assert (oracle.check_tree(g, s, d, q) == []) == (oracle.validate(g, s, d, q) == [])
