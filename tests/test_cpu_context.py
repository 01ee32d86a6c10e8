"""The OpenMP versions of the paper's CPU kernels (BFS-Conventional,
BFS-NonAtomic, BFS-Hybrid with the 5 % rule, BFS-Hybrid dagger,
BFS-VisitedBitmap) give the oracle's distances and valid parents, with one
and several threads, on graphs that take both directions and on deep ones;
the direction rules take the oracle's replayed schedules."""
import numpy as np
import pytest

import cpu_context
import graphgen
import oracle
from tests import graphs

GRAPHS = {
    "rmat12": lambda: graphgen.rmat(12),
    "rmat14": lambda: graphgen.rmat(14),
    "grid64": lambda: graphgen.grid(64),
    "path300": lambda: graphs.path(300)[0],
    "two_paths": lambda: graphs.two_paths(40, 30)[0],
    "urand": lambda: graphgen.urand(1 << 12, 8),
}


@pytest.fixture(scope="module", autouse=True)
def built():
    cpu_context.build(force=True)


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("kind", sorted(cpu_context.KINDS))
def test_matches_oracle(name, kind):
    g = GRAPHS[name]()
    for s in list(graphgen.sources(g, 3, seed=4)) + [0]:
        od = oracle.bfs(g, int(s), want_parent=False)[0]
        for threads in (1, 4):
            d, p, secs, levels = cpu_context.bfs(g, int(s), kind, threads)
            assert np.array_equal(d, od), (name, kind, s, threads)
            assert oracle.validate(g, int(s), d, p, check_component=True) == []
            assert levels == int(od.max()) + 1
            assert secs > 0


def test_hybrid_any_alpha():
    """The direction rule changes only the schedule (alpha = 1 leaves
    top-down only once the frontier holds more edges than the unvisited
    rest, a large alpha after the first level); the distances stay the
    oracle's."""
    g = graphgen.rmat(14)
    s = int(graphgen.sources(g, 1)[0])
    od = oracle.bfs(g, s, want_parent=False)[0]
    for alpha in (1, 14, 1000):
        d, _, _, _ = cpu_context.bfs(g, s, "hybrid_dagger", 4, want_parent=False, alpha=alpha)
        assert np.array_equal(d, od)


def test_rules_take_the_replayed_schedule():
    """With one thread there are no duplicates, so the 5 % rule's
    bottom-up levels are exactly the levels whose frontier holds 5 % of the
    vertices (the oracle's replay), and every frontier entry is distinct."""
    g = graphgen.rmat(14)
    for s in graphgen.sources(g, 3, seed=2):
        od = oracle.bfs(g, int(s), want_parent=False)[0]
        st = oracle.level_stats(g, od)
        for kind in ("hybrid", "visited_bitmap", "nonatomic", "conventional"):
            d, _, _, levels, entries = cpu_context.bfs(g, int(s), kind, 1, want_parent=False,
                                                        return_entries=True)
            assert np.array_equal(d, od) and levels == st["depth"]
            assert entries == st["reached"], (kind, entries, st["reached"])
        sched = oracle.replay_policy(st, oracle.POLICY_FRONTIER_5PCT)
        assert oracle.BU in sched  # the graph does switch


def test_nonatomic_duplicates_counted():
    """Several threads on a lattice: the plain test may admit a vertex more
    than once (never fewer entries than distinct vertices), distances stay
    the oracle's."""
    g = graphgen.grid(256)
    s = int(graphgen.sources(g, 1)[0])
    od = oracle.bfs(g, s, want_parent=False)[0]
    d, p, _, _, entries = cpu_context.bfs(g, s, "nonatomic", 8, return_entries=True)
    assert np.array_equal(d, od)
    assert entries >= int((od >= 0).sum())
    assert oracle.validate(g, s, d, p) == []
