"""The OpenMP versions of the paper's CPU kernels (BFS-Conventional,
BFS-Hybrid dagger, BFS-VisitedBitmap) give the oracle's distances and valid
parents, with one and several threads, on graphs that take both directions
and on deep ones."""
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
        d, _, _, _ = cpu_context.bfs(g, s, "hybrid", 4, want_parent=False, alpha=alpha)
        assert np.array_equal(d, od)
