"""bfs_run_batch_noalloc (the batched search with the library's fixed
per-GPU scratch array) against bfs_run_batch and the oracle: two calls in a
row through the C interface, the second on a smaller input (fewer vertices
and fewer sources, so the array still holds the first call's larger
contents), then a graph too large for the array is refused."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs
from tests.gpu_util import library, say, upload

pytestmark = pytest.mark.gpu


def _rows(bfs, fn, gh, sources):
    import torch
    out = torch.full((len(sources), gh.n), 7, dtype=torch.uint8, device="cuda")
    fn(gh, np.asarray(sources, np.int32), out)
    return out.cpu().numpy()


def test_noalloc_matches_batch_twice():
    bfs = library()
    cases = [(graphgen.rmat(16), 64), (graphgen.rmat(12), 5)]  # the second smaller in n and k
    for g, k in cases:
        say("noalloc batch", g.name, "k", k)
        gh = upload(g)
        srcs = graphgen.sources(g, k)
        got = _rows(bfs, bfs.bfs_run_batch_noalloc, gh, srcs)
        ref = _rows(bfs, bfs.bfs_run_batch, gh, srcs)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(got, oracle.msbfs_dist8(g, [int(s) for s in srcs]))
        gh.close()


def test_noalloc_deep_and_hub_first():
    """A 600-vertex path (distances past 255 saturate) with bit planes
    (k >= 16), and a graph created with hub-first rows and tuned
    parameters, as the benchmark creates its graphs."""
    import bench
    bfs = library()
    g, _ = graphs.path(600)
    gh = upload(g)
    srcs = [0, 599, 300] + list(range(1, 600, 40))
    say("noalloc batch path600 k", len(srcs))
    got = _rows(bfs, bfs.bfs_run_batch_noalloc, gh, srcs)
    np.testing.assert_array_equal(got, oracle.msbfs_dist8(g, srcs))
    gh.close()
    g2 = graphgen.rmat(18)
    gh2, _ = bench.make_handle(bfs, g2)
    srcs2 = graphgen.sources(g2, 64)
    say("noalloc batch rmat18 hub-first k 64")
    got2 = _rows(bfs, bfs.bfs_run_batch_noalloc, gh2, srcs2)
    np.testing.assert_array_equal(got2, _rows(bfs, bfs.bfs_run_batch, gh2, srcs2))
    gh2.close()


def test_noalloc_refuses_graph_beyond_array():
    import torch
    bfs = library()
    n = bfs.BFS_NOALLOC_SCRATCH_BYTES // 88 + 4096  # three sets and eight planes per vertex: too large for k >= 16
    g, _ = graphs.path(n)
    gh = upload(g)
    out = torch.empty((16, n), dtype=torch.uint8, device="cuda")
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_run_batch_noalloc(gh, np.arange(16, dtype=np.int32), out)
    assert e.value.code == bfs.BFS_ERR_INVALID_ARG and "bfs_run_batch" in str(e.value)
    gh.close()
