"""Hub-first rows (BFS_SORT_NEIGHBORS): the device copy of every row equals
the CPU reference order (descending neighbour degree, ties by ascending id,
tests/gpu_util.hub_first) exactly, for rows in each of the sort's length
classes (a wavefront per row up to 64 entries, a workgroup tile up to 4096,
runs merged in global memory beyond), with int64 and int32 row offsets; the
search on such a graph still gives the oracle's distances."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_util import check_single, hub_first, library, say, upload

pytestmark = pytest.mark.gpu


def hub_graph(seed=3):
    """Random background (average degree about 4) plus vertices whose rows
    have exactly the class boundaries' lengths and a few long hubs."""
    rng = np.random.default_rng(seed)
    n = 300_000
    u = [rng.integers(100, n, 600_000)]  # (the listed vertices get only their own rows)
    v = [rng.integers(100, n, 600_000)]
    for hub, deg in enumerate([200_000, 70_001, 8_193, 4_097, 4_096, 65, 64, 63, 2]):
        t = rng.choice(np.arange(100, n), size=deg, replace=False)
        u.append(np.full(deg, hub))
        v.append(t)
    return graphgen.from_edges(n, np.concatenate(u), np.concatenate(v), "hubs")


@pytest.fixture(scope="module")
def bfs():
    return library()


CASES = {"hubs": hub_graph, "rmat16": lambda: graphgen.rmat(16), "rmat20": lambda: graphgen.rmat(20),
         "grid256": lambda: graphgen.grid(256)}


@pytest.mark.parametrize("rp32", [False, True])
@pytest.mark.parametrize("name", sorted(CASES))
def test_rows_in_hub_first_order(bfs, name, rp32):
    g = CASES[name]()
    if name == "hubs":
        assert g.degree[:9].tolist() == [200_000, 70_001, 8_193, 4_097, 4_096, 65, 64, 63, 2]
    say("reorder", name, "rp32", rp32, "max degree", int(g.degree.max()))
    gh = upload(g, bfs.BFS_SORT_NEIGHBORS | (bfs.BFS_ROWPTR32 if rp32 else 0))
    rp, col = bfs.bfs_graph_copy_csr(gh)
    ref = hub_first(g)
    np.testing.assert_array_equal(rp, g.row_ptr)
    if not np.array_equal(col, ref.col_idx):
        bad = np.flatnonzero(col != ref.col_idx)
        row = int(np.searchsorted(g.row_ptr, bad[0], side="right") - 1)
        raise AssertionError(f"{len(bad)} entries out of order, first in row {row} "
                             f"(length {int(g.degree[row])})")
    s = int(graphgen.sources(g, 1)[0])
    check_single(g, gh, s, scan_order=ref)
    gh.close()


def test_copy_csr_unsorted_is_the_input(bfs):
    g = graphgen.rmat(12)
    gh = upload(g)
    rp, col = bfs.bfs_graph_copy_csr(gh)
    np.testing.assert_array_equal(rp, g.row_ptr)
    np.testing.assert_array_equal(col, g.col_idx)
    gh.close()
    assert oracle is not None
