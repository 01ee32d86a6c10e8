"""GPU parity at the full workload sizes, every source compared bit for bit.

The oracle's distances for every source of every full-size workload are
stored as SHA-256 digests with their per-level statistics
(tests/golden/digests.json, written by tests/golden/make_digests.py from the
oracle alone).  Each GPU search here is hashed and compared with its digest;
its per-level frontier sizes, degree sums and direction schedule must equal
the oracle's replay, and its parent array must pass the tree check (every
parent a neighbour one level up).

Configurations:
  * "bench": the graph exactly as bench.py creates it for its timed runs
    (hub-first rows, the autotuned parameters of its graph class), with the
    level loop those parameters select (the captured loop at RMAT scale 24,
    the persistent top-down kernel on the lattice) and with the host-driven
    loop of the instrumented pass;
  * "default": flags 0 and default parameters;
  * RMAT scale 24 also in the benchmark's configuration with the paper's
    alpha = 14, beta = 24 (more hub-heavy levels stay top-down), with the
    5 % frontier rule, and top-down only in the captured loop and in the
    persistent kernel (every hub level expanded top-down).
Workloads: RMAT scale 24 (int64 row offsets, 64 sources), the 4096 x 4096
perturbed lattice (16 sources) and RMAT scale 16 (int32 row offsets, 16
sources)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import bench
import graphgen
import oracle
from tests.gpu_util import (check_graph_digest, check_run_against_digest, golden, library, say,
                            upload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bfs():
    return library()


_GRAPHS = {}


def workload(name):
    if name not in _GRAPHS:
        _GRAPHS.clear()  # one full-size graph in host memory at a time
        say("generating", name)
        g, srcs, rp32 = bench.make_graph(name)
        rec = golden()[name]
        check_graph_digest(g, rec["graph"])
        assert [int(s) for s in srcs] == rec["sources"]
        _GRAPHS[name] = (g, srcs, rp32, rec)
    return _GRAPHS[name]


def run_all(bfs, g, gh, rec, parents, pool):
    """Every source of the record: digest, statistics, schedule; parent
    trees checked on the host in `pool` while the GPU runs the next ones."""
    import torch
    params = bfs.bfs_get_params(gh)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    par = torch.empty(g.n, dtype=torch.int32, device="cuda") if parents else None
    checks = []
    for r in rec["runs"]:
        s = r["source"]
        bfs.bfs_run(gh, s, dist, par)
        run, levels = bfs.bfs_get_run_stats(gh)
        d = dist.cpu().numpy()
        check_run_against_digest(r, d, run, levels, params, g.n, g.nnz)
        if parents:
            p = par.cpu().numpy()
            checks.append((s, pool.submit(oracle.check_tree, g, s, d, p)))
    for s, f in checks:
        assert f.result() == [], (s, f.result())
    return len(rec["runs"])


CASES = [("rmat24", "bench", None), ("rmat24", "bench", "host"), ("rmat24", "bench", "alpha14"),
         ("rmat24", "bench", "pct5"), ("rmat24", "bench", "tdonly"), ("rmat24", "bench", "tdonly_persistent"),
         ("rmat24", "default", None),
         ("grid4096", "bench", None), ("grid4096", "bench", "host"), ("grid4096", "default", None),
         ("rmat16", "bench", None), ("rmat16", "bench", "host"), ("rmat16", "default", None)]


@pytest.mark.parametrize("name,config,loop", CASES, ids=[f"{a}-{b}-{c or 'graph'}" for a, b, c in CASES])
def test_every_source(bfs, name, config, loop):
    g, srcs, rp32, rec = workload(name)
    if config == "bench":
        gh, _ = bench.make_handle(bfs, g, rp32)
    else:
        gh = upload(g, bfs.BFS_ROWPTR32 if rp32 else 0)
    info = bfs.bfs_graph_info_get(gh)
    assert info["row_ptr_bytes"] == (4 if rp32 else 8) and info["nnz"] == g.nnz
    if loop == "host":
        bfs.bfs_set_params(gh, loop=bfs.BFS_LOOP_HOST, collect_timing=1)
    elif loop == "alpha14":
        # the paper's alpha / beta: more hub-heavy levels stay top-down, and
        # those skip the frontier summary (checked against the same replay)
        bfs.bfs_set_params(gh, policy=1, alpha=14, beta=24)
    elif loop == "pct5":
        bfs.bfs_set_params(gh, policy=2)  # the 5 % frontier rule
    elif loop == "tdonly":
        bfs.bfs_set_params(gh, policy=3)  # every hub level through the per-chunk role
    elif loop == "tdonly_persistent":
        bfs.bfs_set_params(gh, policy=3, loop=bfs.BFS_LOOP_PERSISTENT)
    say(name, config, loop or "graph", "params", bfs.bfs_get_params(gh))
    # parents of every source in the benchmark's own configuration
    with ThreadPoolExecutor(8) as pool:
        done = run_all(bfs, g, gh, rec, parents=(config == "bench"), pool=pool)
    assert done == len(srcs)
    run, _ = bfs.bfs_get_run_stats(gh)
    # the host loop when asked for, else the handle's loop (the tuned one in the
    # benchmark's configuration; AUTO runs the captured loop)
    tuned_loop = bfs.bfs_get_params(gh)["loop"]
    expect_loop = bfs.BFS_LOOP_HOST if loop == "host" else (tuned_loop or bfs.BFS_LOOP_GRAPH)
    if loop == "alpha14":
        assert run["policy"] == 1
    elif loop in ("pct5", "tdonly", "tdonly_persistent"):
        assert run["policy"] == (2 if loop == "pct5" else 3)
    if loop == "tdonly_persistent":
        expect_loop = bfs.BFS_LOOP_PERSISTENT
    assert run["loop"] == expect_loop
    gh.close()
