"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (default tunables):
  * RMAT scale 24, edge factor 16, int64 row offsets, 64 sources;
  * 4096 x 4096 perturbed lattice (10 % deletion, 1 % shortcuts), 16 sources.
A few sources are compared with the oracle in full (bit-exact distances,
per-level schedule and work); every source is checked on a sample of
vertices against local BFS properties and on its reached count against the
connected component of its source."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_util import check_single, gpu_bfs, library, say, upload

pytestmark = pytest.mark.gpu


def _component_sizes(g):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    a = csr_matrix((np.ones(g.nnz, np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(a, directed=False)
    return lab, np.bincount(lab)


def _sampled_checks(g, s, d, p, rng, k=20000):
    """For sampled vertices v: neighbours within one level; a reached v != s
    has a neighbour one level up and its parent is such a neighbour; an
    unreached v has only unreached neighbours."""
    assert d[s] == 0 and p[s] == s
    vs = rng.integers(0, g.n, k)
    rp, col = g.row_ptr, g.col_idx
    for v in vs:
        nb = col[rp[v]:rp[v + 1]]
        dn = d[nb]
        if d[v] < 0:
            assert (dn < 0).all() and p[v] == -1
        elif v != s:
            assert (dn >= 0).all() and (np.abs(dn - d[v]) <= 1).all()
            assert (dn == d[v] - 1).any()
            assert p[v] in nb and d[p[v]] == d[v] - 1


@pytest.fixture(scope="module")
def bfs():
    return library()


@pytest.fixture(scope="module")
def rmat24():
    say("generating rmat24")
    return graphgen.rmat(24)


@pytest.fixture(scope="module")
def grid4096():
    say("generating grid4096")
    return graphgen.grid(4096)


def test_rmat24(bfs, rmat24):
    g = rmat24
    gh = upload(g)  # int64 row offsets
    info = bfs.bfs_graph_info_get(gh)
    assert info["row_ptr_bytes"] == 8 and info["nnz"] == g.nnz
    srcs = graphgen.sources(g, 64)
    lab, sizes = _component_sizes(g)
    for i, s in enumerate(srcs[:2]):
        say("rmat24 full parity source", s)
        check_single(g, gh, s, full_validate=(i == 0))
    rng = np.random.default_rng(0)
    for s in srcs:
        say("rmat24 sampled source", s)
        d, p = gpu_bfs(gh, s)
        run, levels = bfs.bfs_get_run_stats(gh)
        assert run["reached"] == sizes[lab[s]] == int((d >= 0).sum())
        _sampled_checks(g, s, d, p, rng, k=2000)
    gh.close()


def test_grid4096(bfs, grid4096):
    g = grid4096
    gh = upload(g)
    srcs = graphgen.sources(g, 16)
    lab, sizes = _component_sizes(g)
    for i, s in enumerate(srcs[:3]):
        say("grid4096 full parity source", s)
        _, _, run, _ = check_single(g, gh, s, full_validate=(i == 0))
        assert run["loop"] == bfs.BFS_LOOP_GRAPH and run["levels"] > 1000
    rng = np.random.default_rng(1)
    for s in srcs:
        say("grid4096 sampled source", s)
        d, p = gpu_bfs(gh, s)
        run, _ = bfs.bfs_get_run_stats(gh)
        assert run["reached"] == sizes[lab[s]] == int((d >= 0).sum())
        _sampled_checks(g, s, d, p, rng, k=2000)
    gh.close()
