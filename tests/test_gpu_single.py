"""GPU parity of the single-source search (bfs_run) against the oracle.

Distances must be bit-exact; parents must satisfy the BFS-tree invariants
(they may differ from the oracle's); per-level frontier sizes, the direction
schedule and the bottom-up work counts must equal the oracle's replay of the
same switching rule."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs
from tests.gpu_util import check_single, gpu_bfs, hub_first, library, say, upload

pytestmark = pytest.mark.gpu

POLICIES = {"alpha_beta": 1, "frontier_5pct": 2, "td_only": 3}


@pytest.fixture(scope="module")
def bfs():
    return library()


@pytest.mark.parametrize("name", sorted(graphs.CLOSED_FORMS))
@pytest.mark.parametrize("policy", sorted(POLICIES))
@pytest.mark.parametrize("loop", [1, 2, 3, 4])
def test_closed_forms(bfs, name, policy, loop):
    g, f = graphs.CLOSED_FORMS[name]()
    say("closed form", name, policy, "loop", loop)
    gh = upload(g)
    bfs.bfs_set_params(gh, policy=POLICIES[policy], loop=loop, graph_chunk_levels=5)
    srcs = [0] if name == "binary_tree" else sorted({0, g.n // 3, g.n - 1})
    for s in srcs:
        d, _, _, _ = check_single(g, gh, s, ref=f(s).astype(np.int32))
    gh.close()


@pytest.fixture(scope="module")
def rmat16():
    return graphgen.rmat(16)


def test_rmat16_config(bfs, rmat16):
    """RMAT scale 16, edge factor 16, int32 row offsets, 16 sources, default
    (auto = alpha/beta) policy."""
    g = rmat16
    say("rmat16 int32 row_ptr, 16 sources")
    gh = upload(g, bfs.BFS_ROWPTR32)
    assert bfs.bfs_graph_info_get(gh)["row_ptr_bytes"] == 4
    for s in graphgen.sources(g, 16):
        _, _, run, levels = check_single(g, gh, s)
        assert run["policy"] == bfs.BFS_POLICY_ALPHA_BETA
    gh.close()


@pytest.mark.parametrize("policy", sorted(POLICIES))
@pytest.mark.parametrize("loop", [1, 2, 4])
@pytest.mark.parametrize("rp32", [False, True])
def test_rmat16_policies_loops(bfs, rmat16, policy, loop, rp32):
    g = rmat16
    say("rmat16", policy, "loop", loop, "rp32", rp32)
    gh = upload(g, bfs.BFS_ROWPTR32 if rp32 else 0)
    bfs.bfs_set_params(gh, policy=POLICIES[policy], loop=loop, graph_chunk_levels=3)
    for s in graphgen.sources(g, 4, seed=77):
        check_single(g, gh, s)
    gh.close()


@pytest.mark.parametrize("t1,t2,tbu,bs", [(1, 64, 1, 64), (2, 100, 4, 128), (8, 256, 16, 1024),
                                          (1000, 100000, 100000, 256), (32, 2048, 64, 512)])
def test_threshold_sweep(bfs, rmat16, t1, t2, tbu, bs):
    """Every degree bucket and both bottom-up paths, across workgroup sizes."""
    g = rmat16
    say("rmat16 thresholds", t1, t2, tbu, bs)
    gh = upload(g)
    bfs.bfs_set_params(gh, td_wave_degree=t1, td_block_degree=t2, bu_wave_degree=tbu, block_size=bs)
    for pol in (1, 2):
        bfs.bfs_set_params(gh, policy=pol)
        for s in graphgen.sources(g, 3, seed=11):
            check_single(g, gh, s)
    gh.close()


@pytest.mark.parametrize("loop", [1, 2, 3])
def test_large_queue_windows(bfs, rmat16, loop):
    """Top-down-only searches with a low large-vertex threshold (t2 = 64) and
    64-thread workgroups: a level queues hundreds of large vertices (one
    entry each, with its chunk count), which the large role reads in many
    64-entry windows and splits into chunks round-robin over its
    workgroups; distances, parents and every level record equal the
    oracle's, in the host, captured and persistent loops."""
    g = rmat16
    say("rmat16 large-queue windows, loop", loop)
    gh = upload(g)
    bfs.bfs_set_params(gh, policy=3, loop=loop, td_wave_degree=8, td_block_degree=64, block_size=64,
                       graph_td_blocks=16)
    for s in graphgen.sources(g, 3, seed=21):
        check_single(g, gh, s)
    gh.close()


def test_repeat_identical(bfs, rmat16):
    g = rmat16
    say("rmat16 repeat x20")
    gh = upload(g)
    s = int(graphgen.sources(g, 1)[0])
    ref, _ = gpu_bfs(gh, s)
    for _ in range(20):
        d, p = gpu_bfs(gh, s)
        assert np.array_equal(d, ref)
        assert oracle.validate(g, s, d, p, check_component=False) == []
    gh.close()


def test_edge_cases(bfs):
    say("edge cases")
    # single vertex
    g1 = graphgen.from_edges(1, [], [])
    gh = upload(g1)
    d, p = gpu_bfs(gh, 0)
    assert d.tolist() == [0] and p.tolist() == [0]
    gh.close()
    # no edges at all, several vertices
    g0 = graphgen.from_edges(70, [], [])
    gh = upload(g0)
    d, p = gpu_bfs(gh, 69)
    assert d[69] == 0 and (np.delete(d, 69) == -1).all() and p[69] == 69
    gh.close()
    # isolated source inside a connected graph
    g, _ = graphs.path(100)
    gi = graphgen.from_edges(101, *[np.arange(99), np.arange(1, 100)])
    gh = upload(gi)
    check_single(gi, gh, 100)
    check_single(gi, gh, 0)
    gh.close()
    # n not a multiple of 64, last word partly used
    gr = graphs.random_graph(130, 400, 3)
    gh = upload(gr)
    for s in (0, 64, 129):
        check_single(gr, gh, s)
    gh.close()


@pytest.mark.parametrize("loop", [1, 2, 3, 4])
def test_hub_chunks(bfs, loop):
    """A hub of degree 50 000 (far above td_block_degree) as source and as a
    discovered vertex: its row is split into workgroup chunks."""
    say("hub chunks loop", loop)
    k = 50000
    u = np.concatenate([np.zeros(k, np.int64), np.arange(1, 200)])
    v = np.concatenate([np.arange(1, k + 1), np.arange(2, 201)])
    g = graphgen.from_edges(k + 1, u, v)
    gh = upload(g)
    bfs.bfs_set_params(gh, loop=loop, policy=3, td_block_degree=1024)
    for s in (0, 1, 150, k):
        check_single(g, gh, s)
    bfs.bfs_set_params(gh, policy=1)
    for s in (0, 150):
        check_single(g, gh, s)
    gh.close()


@pytest.mark.parametrize("k", [1, 7, 32, 4096])
def test_long_path_graph_loop(bfs, k):
    """Thousands of levels through the captured level loop, chunk sizes that
    do and do not divide the level count."""
    say("path 3000, graph chunk", k)
    g, f = graphs.path(3000)
    gh = upload(g)
    bfs.bfs_set_params(gh, loop=2, policy=3, graph_chunk_levels=k)
    check_single(g, gh, 0, ref=f(0).astype(np.int32))
    check_single(g, gh, 1500, ref=f(1500).astype(np.int32))
    gh.close()


def test_device_input(bfs, rmat16):
    import torch
    g = rmat16
    say("device-resident CSR input")
    rp = torch.from_numpy(g.row_ptr.copy()).cuda()
    col = torch.from_numpy(g.col_idx.copy()).cuda()
    gh = bfs.bfs_create_graph(rp, col, bfs.BFS_VALIDATE)
    check_single(g, gh, int(graphgen.sources(g, 1)[0]))
    gh.close()


def test_validate_flags(bfs):
    say("create-time validation")
    rp = np.array([0, 1, 1], np.int64)
    col = np.array([1], np.int32)  # 0->1 without 1->0
    with pytest.raises(bfs.BfsError):
        bfs.bfs_create_graph(rp, col, bfs.BFS_VALIDATE | bfs.BFS_VALIDATE_SYMMETRY)
    with pytest.raises(bfs.BfsError):
        bfs.bfs_create_graph(np.array([0, 1, 2], np.int64), np.array([1, 5], np.int32), bfs.BFS_VALIDATE)
    gh = bfs.bfs_create_graph(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32),
                              bfs.BFS_VALIDATE | bfs.BFS_VALIDATE_SYMMETRY)
    import torch
    d = torch.empty(2, dtype=torch.int32, device="cuda")
    with pytest.raises(bfs.BfsError):
        bfs.bfs_run(gh, 2, d)
    with pytest.raises(bfs.BfsError):
        bfs.bfs_set_params(gh, block_size=100)
    for bad in ({"queue_ahead": 65}, {"queue_ahead": -1}, {"bu_blocks": 1025}, {"loop": 5}):
        with pytest.raises(bfs.BfsError):
            bfs.bfs_set_params(gh, **bad)
    gh.close()


def test_grid_small_many_sources(bfs):
    """512 x 512 perturbed lattice (average degree 3.6 => auto picks top-down
    only and the captured level loop)."""
    g = graphgen.grid(512)
    say("grid512, 8 sources")
    gh = upload(g)
    for s in graphgen.sources(g, 8):
        _, _, run, _ = check_single(g, gh, s)
        assert run["policy"] == 3 and run["loop"] == bfs.BFS_LOOP_GRAPH
    gh.close()


def test_urand(bfs):
    g = graphgen.urand(1 << 16, 16)
    say("urand 2^16 d16")
    gh = upload(g)
    for s in graphgen.sources(g, 4):
        check_single(g, gh, s)
    gh.close()


@pytest.mark.parametrize("rp32", [False, True])
def test_sorted_neighbours(bfs, rmat16, rp32):
    """BFS_SORT_NEIGHBORS: distances unchanged; bottom-up work equals the
    oracle's profile on the hub-first order."""
    g = rmat16
    say("rmat16 hub-first rows, rp32", rp32)
    flags = bfs.BFS_SORT_NEIGHBORS | (bfs.BFS_ROWPTR32 if rp32 else 0)
    gh = upload(g, flags)
    order = hub_first(g)
    for pol in (1, 2):
        bfs.bfs_set_params(gh, policy=pol)
        for s in graphgen.sources(g, 4, seed=123):
            check_single(g, gh, s, scan_order=order)
    gh.close()
    # a graph with ties and isolated vertices
    gr = graphs.random_graph(3000, 9000, 8)
    gh = upload(gr, bfs.BFS_SORT_NEIGHBORS)
    for s in (0, 1500, 2999):
        check_single(gr, gh, s, scan_order=hub_first(gr))
    gh.close()


@pytest.mark.parametrize("blocks", [1, 2, 3, 16, 128, 512])
def test_persistent_loop_grid_sizes(bfs, rmat16, blocks):
    """The persistent top-down loop with grids from one workgroup upward, on a
    long path (thousands of levels) and on RMAT (every degree class)."""
    say("persistent loop, blocks", blocks)
    g, f = graphs.path(2500)
    gh = upload(g)
    bfs.bfs_set_params(gh, loop=3, policy=3, graph_td_blocks=blocks)
    _, _, run, _ = check_single(g, gh, 7, ref=f(7).astype(np.int32))
    assert run["loop"] == 3
    gh.close()
    gh = upload(rmat16)
    bfs.bfs_set_params(gh, loop=3, policy=3, graph_td_blocks=blocks, td_block_degree=256)
    if blocks < 3:
        with pytest.raises(bfs.BfsError):  # three degree classes need three roles
            gpu_bfs(gh, int(graphgen.sources(rmat16, 1)[0]))
    else:
        for s in graphgen.sources(rmat16, 2, seed=5):
            check_single(rmat16, gh, s)
    gh.close()


@pytest.mark.parametrize("bs,bu_blocks", [(64, 1), (64, 3), (128, 2), (512, 0)])
def test_bu_runs_of_many_words(bs, bu_blocks):
    """Bottom-up grids far smaller than the word count, so each wavefront
    takes several 64-word runs of many 64-candidate batches: deferred rows
    pile up to the ring's limit and the last batch of a run leaves more
    than 64 of them to scan."""
    bfs = library()
    say("bottom-up runs: block", bs, "bu_blocks", bu_blocks)
    g, f = graphs.deferred_rows()
    gh = upload(g)
    bfs.bfs_set_params(gh, policy=2, block_size=bs, bu_blocks=bu_blocks)
    _, _, run, levels = check_single(g, gh, 0, ref=f(0).astype(np.int32))
    assert levels[1]["direction"] == 1 and levels[1]["examined"] > 4 * levels[1]["scanned"] // 2
    gh.close()


@pytest.mark.parametrize("bu_blocks", [1, 5, 64])
@pytest.mark.parametrize("sort", [False, True])
def test_rmat16_bu_blocks(rmat16, bu_blocks, sort):
    bfs = library()
    g = rmat16
    say("rmat16 bu_blocks", bu_blocks, "sorted", sort)
    gh = upload(g, bfs.BFS_SORT_NEIGHBORS if sort else 0)
    bfs.bfs_set_params(gh, block_size=64, bu_blocks=bu_blocks)
    order = hub_first(g) if sort else None
    for pol in (1, 2):
        bfs.bfs_set_params(gh, policy=pol)
        for s in graphgen.sources(g, 3, seed=19):
            check_single(g, gh, s, scan_order=order)
    gh.close()


@pytest.mark.parametrize("policy", [1, 3])
@pytest.mark.parametrize("loop,ahead", [(1, 2), (4, 1), (4, 2), (4, 16)])
def test_level_timing(rmat16, policy, loop, ahead):
    """collect_timing: every level of a host-loop or queued-loop run gets a
    device time (queued lookahead shorter and longer than the search)."""
    bfs = library()
    g = rmat16
    say("rmat16 level timing, policy", policy, "loop", loop, "ahead", ahead)
    gh = upload(g)
    bfs.bfs_set_params(gh, policy=policy, loop=loop, queue_ahead=ahead, collect_timing=1)
    for s in graphgen.sources(g, 4, seed=29):
        _, _, run, levels = check_single(g, gh, s)
        assert run["loop"] == loop and all(lv["ms"] > 0 for lv in levels), levels
    gh.close()


@pytest.fixture(scope="module")
def rmat20():
    return graphgen.rmat(20)


@pytest.fixture(scope="module")
def rmat20_hub_first(rmat20):
    return hub_first(rmat20)


@pytest.mark.parametrize("policy", [1, 2])
@pytest.mark.parametrize("sort", [False, True])
def test_rmat20_repeated_full_parity(rmat20, rmat20_hub_first, policy, sort):
    """RMAT scale 20 (a million vertices: every wavefront of the level
    kernels busy at once), hybrid policies whose schedules switch back to
    top-down, each source run three times, every run compared in full with
    the oracle.  Races between wavefronts of one level show up here as runs
    that differ."""
    bfs = library()
    g = rmat20
    say("rmat20 repeated parity, policy", policy, "sorted", sort)
    gh = upload(g, bfs.BFS_SORT_NEIGHBORS if sort else 0)
    bfs.bfs_set_params(gh, policy=policy)
    order = rmat20_hub_first if sort else None
    for s in graphgen.sources(g, 6, seed=41):
        ref = oracle.bfs(g, s, want_parent=False)[0]
        for rep in range(3):
            check_single(g, gh, s, ref=ref, full_validate=(rep == 0), scan_order=order)
    gh.close()


@pytest.mark.parametrize("loop", [1, 2, 3, 4])
def test_td_visited_dist_cas(rmat16, loop):
    """The paper's BFS-Conventional visited test (compare-and-swap on the
    distance, no bitmap): distances, parents and every level statistic as
    the oracle's top-down-only replay."""
    bfs = library()
    say("td_visited dist_cas, loop", loop)
    for name, g in (("rmat16", rmat16), ("grid256", graphgen.grid(256)), ("path500", graphs.path(500)[0])):
        gh = upload(g)
        bfs.bfs_set_params(gh, policy=3, loop=loop, td_visited=bfs.BFS_TD_DIST_CAS)
        for s in graphgen.sources(g, 3, seed=7):
            say("  graph", name, "source", int(s))
            check_single(g, gh, s)
        gh.close()


def _check_plain(bfs, g, gh, s, overflow_ok=False):
    """Distances of a plain-visited-test search bit-exact, parents valid,
    per-level frontiers at least the oracle's.  With `overflow_ok` the
    search may instead stop with the documented queue-overflow error."""
    try:
        d, p = gpu_bfs(gh, s)
    except bfs.BfsError as e:
        assert overflow_ok and e.code == bfs.BFS_ERR_OUT_OF_MEMORY, e
        assert "appended more frontier entries than the queues hold" in str(e)
        return False
    od = oracle.bfs(g, s, want_parent=False)[0]
    assert np.array_equal(d, od)
    assert oracle.validate(g, s, d, p, check_component=True) == []
    run, levels = bfs.bfs_get_run_stats(gh)
    st = oracle.level_stats(g, od)
    assert run["levels"] == st["depth"] and run["reached"] >= st["reached"]
    nf = np.array([lv["frontier"] for lv in levels])
    assert nf[0] == 1 and (nf >= st["h"]).all()
    assert all(lv["direction"] == 0 for lv in levels)
    return True


@pytest.mark.parametrize("loop", [1, 2, 3, 4])
def test_td_visited_dist_plain(rmat16, loop):
    """The paper's BFS-NonAtomic visited test (plain test and store of the
    distance): distances bit-exact and parents valid; racing discoverers may
    append a vertex more than once, so each level's frontier is at least the
    oracle's and the level count is the same.  Every copy is expanded, so on
    the lattice the copies can multiply along shortest paths until the
    queues are full: there the search must either finish exact or stop with
    the overflow error (never write past a queue)."""
    bfs = library()
    say("td_visited dist_plain, loop", loop)
    for g, lattice in ((rmat16, False), (graphgen.grid(256), True), (graphs.path(500)[0], False)):
        gh = upload(g)
        bfs.bfs_set_params(gh, policy=3, loop=loop, td_visited=bfs.BFS_TD_DIST_PLAIN)
        for s in graphgen.sources(g, 3, seed=7):
            _check_plain(bfs, g, gh, s, overflow_ok=lattice)
        # the handle stays usable after an overflow
        bfs.bfs_set_params(gh, td_visited=bfs.BFS_TD_VISITED_BITMAP)
        check_single(g, gh, int(graphgen.sources(g, 1, seed=8)[0]))
        gh.close()


@pytest.mark.parametrize("loop", [1, 2, 3, 4])
def test_td_visited_dist_plain_cull(rmat16, loop):
    """The plain visited test with duplicate copies culled at expansion
    (only the copy whose position the last appender recorded expands):
    exact distances on every graph, the lattice included."""
    bfs = library()
    say("td_visited dist_plain_cull, loop", loop)
    for g in (rmat16, graphgen.grid(256), graphs.path(500)[0], graphs.deferred_rows()[0]):
        gh = upload(g)
        bfs.bfs_set_params(gh, policy=3, loop=loop, td_visited=bfs.BFS_TD_DIST_PLAIN_CULL)
        for s in graphgen.sources(g, 3, seed=7):
            assert _check_plain(bfs, g, gh, s)
        gh.close()


def test_td_visited_needs_td_only(rmat16):
    bfs = library()
    say("td_visited needs top-down only")
    gh = upload(rmat16)
    bfs.bfs_set_params(gh, policy=1, td_visited=bfs.BFS_TD_DIST_CAS)
    with pytest.raises(bfs.BfsError):
        gpu_bfs(gh, 0)
    bfs.bfs_set_params(gh, td_visited=bfs.BFS_TD_VISITED_BITMAP)
    check_single(rmat16, gh, int(graphgen.sources(rmat16, 1)[0]))
    gh.close()


@pytest.mark.parametrize("loop", [1, 2, 4])
def test_summary_skipped_then_small_bottom_up(bfs, loop):
    """A top-down level that skips the frontier summary (its expected
    frontier is too large for a bottom-up level to test the summary), then
    a bottom-up level with a frontier small enough to test it: the summary
    counts as incomplete, so the level reads the frontier bitmap itself.
    One bottom-up wavefront, so its runs are long enough to hold summary
    bytes (tests/test_oracle_policy.py pins the schedule and sizes on the
    CPU)."""
    g = graphs.summary_skip()
    say("summary skip, loop", loop)
    gh = upload(g)
    bfs.bfs_set_params(gh, policy=1, alpha=75, beta=24, block_size=64, bu_blocks=1, loop=loop)
    _, _, run, levels = check_single(g, gh, 0)
    assert [lv["direction"] for lv in levels] == [0, 0, 0, 1, 1]
    assert levels[3]["frontier"] == 138 and run["reached"] == 1 + 1 + 41 + 138 + 2340
    gh.close()

