"""GPU tests of the serving runtime (continuous batching).

Each request's result must equal the oracle's distances bit for bit, alone
and in a mix of concurrent requests on several graphs, with valid parents
where requested; admission, lane joins during long searches, budget limits
and error paths are exercised from the host."""
import time

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs
from tests.gpu_util import library, say, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bfs():
    return library()


def wait_all(bfs, srv, tickets, timeout=60.0):
    t0 = time.time()
    pending = set(tickets)
    stats = {}
    while pending:
        for t in list(pending):
            state, st = bfs.bfs_serve_poll(srv, t)
            if state in (bfs.BFS_REQ_DONE, bfs.BFS_REQ_FAILED):
                assert state == bfs.BFS_REQ_DONE, f"request {t} failed"
                stats[t] = st
                pending.discard(t)
        if time.time() - t0 > timeout:
            raise TimeoutError(f"{len(pending)} requests still pending")
        time.sleep(0.0005)
    return stats


@pytest.fixture(scope="module")
def pool(bfs):
    gs = {
        "rmat12": graphgen.rmat(12),
        "rmat14": graphgen.rmat(14),
        "grid64": graphgen.grid(64),
        "path700": graphs.path(700)[0],
        "urand4k": graphgen.urand(1 << 12, 8),
        "two_paths": graphs.two_paths(40, 30)[0],
        # a 1000-edge row next to the source: top-down levels expand it in
        # chunks spread over the grid
        "long_row": graphs.deferred_rows(n=4096, nf=1500, seed=5)[0],
    }
    handles = {k: upload(g) for k, g in gs.items()}
    yield gs, handles
    for h in handles.values():
        h.close()


def make_requests(gs, n, seed):
    rng = np.random.default_rng(seed)
    names = sorted(gs)
    reqs = []
    for i in range(n):
        name = names[int(rng.integers(len(names)))]
        g = gs[name]
        nz = np.flatnonzero(g.degree > 0)
        s = int(nz[rng.integers(len(nz))]) if i % 17 else int(rng.integers(g.n))  # some isolated
        reqs.append((name, s, bool(i % 3 == 0)))
    return reqs


def submit(bfs, srv, gs, handles, name, s, want_parent):
    import torch
    n = gs[name].n
    d = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    p = torch.full((n,), -7, dtype=torch.int32, device="cuda") if want_parent else None
    torch.cuda.synchronize()  # the server writes from its own streams
    t = bfs.bfs_serve_submit(srv, handles[name], s, d, p)
    return t, d, p


def check(gs, name, s, d, p):
    g = gs[name]
    od, _ = oracle.bfs(g, s, want_parent=False)
    dn = d.cpu().numpy()
    assert np.array_equal(dn, od), f"{name} source {s}: {(dn != od).sum()} wrong distances"
    if p is not None:
        assert oracle.validate(g, s, dn, p.cpu().numpy(), check_component=False) == []


def test_alone_equals_mix(bfs, pool):
    import torch
    gs, handles = pool
    reqs = make_requests(gs, 120, seed=3)
    srv = bfs.bfs_serve_create(1 << 34, 64)
    say("serve: each request alone")
    alone = []
    for name, s, wp in reqs:
        t, d, p = submit(bfs, srv, gs, handles, name, s, wp)
        wait_all(bfs, srv, [t])
        alone.append(d.cpu().numpy())
        check(gs, name, s, d, p)
    say("serve: all requests in a mix")
    rng = np.random.default_rng(9)
    outs = []
    for i, (name, s, wp) in enumerate(reqs):
        outs.append(submit(bfs, srv, gs, handles, name, s, wp))
        if rng.random() < 0.3:
            time.sleep(float(rng.random()) * 0.002)  # arrivals while others run
    stats = wait_all(bfs, srv, [t for t, _, _ in outs])
    for (name, s, wp), (t, d, p), a in zip(reqs, outs, alone):
        assert np.array_equal(d.cpu().numpy(), a)
        check(gs, name, s, d, p)
        st = stats[t]
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
        od, _ = oracle.bfs(gs[name], s, want_parent=False)
        assert st["levels"] == int(od.max()) + 1
    assert max(st["batch_lanes"] for st in stats.values()) > 1  # requests did share batches
    bfs.bfs_serve_destroy(srv)
    torch.cuda.synchronize()


def test_long_rows_in_chunks(bfs, pool):
    """Sources on and next to rows longer than the server's chunk length,
    alone and sharing a batch."""
    gs, handles = pool
    g = gs["long_row"]
    big = np.flatnonzero(g.degree > 512)
    assert len(big) > 0
    srv = bfs.bfs_serve_create(1 << 34, 64)
    say("serve: long rows in chunks")
    srcs = [0] + [int(x) for x in big[:3]] + [int(g.col_idx[g.row_ptr[int(big[0])]])]
    outs = [submit(bfs, srv, gs, handles, "long_row", s, True) for s in srcs]
    wait_all(bfs, srv, [t for t, _, _ in outs])
    for s, (t, d, p) in zip(srcs, outs):
        check(gs, "long_row", s, d, p)
    bfs.bfs_serve_destroy(srv)


def test_lanes_join_long_search(bfs, pool):
    """Requests submitted while a 700-level search runs join its batch."""
    gs, handles = pool
    srv = bfs.bfs_serve_create(1 << 34, 64)
    say("serve: joins during a long search")
    first = submit(bfs, srv, gs, handles, "path700", 0, True)
    time.sleep(0.001)
    more = [submit(bfs, srv, gs, handles, "path700", s, s % 2 == 0) for s in (699, 350, 10, 600, 1)]
    wait_all(bfs, srv, [first[0]] + [t for t, _, _ in more])
    for s, (t, d, p) in zip([0, 699, 350, 10, 600, 1], [first] + more):
        check(gs, "path700", s, d, p)
    bfs.bfs_serve_destroy(srv)


def test_tight_budget_and_one_lane(bfs, pool):
    gs, handles = pool
    # room for about one batch of the largest pool graph at a time
    srv = bfs.bfs_serve_create(48 * gs["rmat14"].n + (1 << 16), 1)
    say("serve: tight budget, one lane per batch")
    reqs = make_requests(gs, 30, seed=5)
    outs = [submit(bfs, srv, gs, handles, *r) for r in reqs]
    wait_all(bfs, srv, [t for t, _, _ in outs])
    for (name, s, wp), (t, d, p) in zip(reqs, outs):
        check(gs, name, s, d, p)
    bfs.bfs_serve_destroy(srv)


def test_errors(bfs, pool):
    import torch
    gs, handles = pool
    srv = bfs.bfs_serve_create(1024, 64)  # smaller than any batch
    d = torch.empty(gs["rmat12"].n, dtype=torch.int32, device="cuda")
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_serve_submit(srv, handles["rmat12"], 0, d)
    assert e.value.code == 2
    with pytest.raises(bfs.BfsError):
        bfs.bfs_serve_poll(srv, 12345)
    with pytest.raises(bfs.BfsError):
        bfs.bfs_serve_submit(srv, handles["rmat12"], gs["rmat12"].n, d)
    bfs.bfs_serve_destroy(srv)
    with pytest.raises(bfs.BfsError):
        bfs.bfs_serve_create(1 << 30, 65)


def test_destroy_graph_busy(bfs):
    import torch
    g, _ = graphs.path(3000)
    gh = upload(g)
    srv = bfs.bfs_serve_create(1 << 32, 4)
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t = bfs.bfs_serve_submit(srv, gh, 0, d)
    try:
        gh.close()
        closed = True  # the request may already have finished
    except bfs.BfsError as e:
        assert e.code == 4  # BUSY while the request is in the server
        closed = False
    wait_all(bfs, srv, [t])
    bfs.bfs_serve_destroy(srv)
    if not closed:
        gh.close()


def test_pool_at_full_size(bfs):
    """The serving pool at its real sizes (12 graphs: RMAT 14-23, lattices up
    to 2048^2, uniform random graphs of 2^20 vertices), created as the
    benchmark creates them: 4 requests per graph through one server, first
    one per graph alone, then all 48 interleaved under a budget that keeps
    most batches waiting; every distance array equals the oracle's (SHA-256
    digests written from the oracle) and parents form valid trees."""
    import torch

    import bench
    from tests.gpu_util import check_graph_digest, golden, sha256
    rec = golden()["pool"]
    gs, handles = {}, {}
    for kind, size in bench.SERVE_POOL:
        name = f"{kind}{size}"
        say("serve pool: generating", name)
        g = bench._serve_graph(kind, size)
        check_graph_digest(g, rec[name]["graph"])
        gs[name] = g
        handles[name] = bench.make_handle(bfs, g)[0]
    reqs = [(name, r["source"], i % 2 == 0, r["dist_sha256"])
            for i in range(4) for name in gs for r in rec[name]["runs"][i:i + 1]]

    def verify(name, s, d, p, digest):
        dn = d.cpu().numpy()
        assert sha256(dn.astype("<i4")) == digest, f"{name} source {s}: distances differ from the oracle's"
        if p is not None:
            assert oracle.check_tree(gs[name], s, dn, p.cpu().numpy()) == [], (name, s)

    largest = max(36 * g.n for g in gs.values())
    srv = bfs.bfs_serve_create(largest + (256 << 20), 64)
    say("serve pool: alone")
    for name, s, wp, digest in reqs[:len(gs)]:
        t, d, p = submit(bfs, srv, gs, handles, name, s, wp)
        wait_all(bfs, srv, [t], timeout=120.0)
        verify(name, s, d, p, digest)
    say("serve pool: 48 requests interleaved")
    outs = [submit(bfs, srv, gs, handles, name, s, wp) for name, s, wp, _ in reqs]
    wait_all(bfs, srv, [t for t, _, _ in outs], timeout=120.0)
    for (name, s, wp, digest), (t, d, p) in zip(reqs, outs):
        verify(name, s, d, p, digest)
    bfs.bfs_serve_destroy(srv)
    torch.cuda.synchronize()
    for h in handles.values():
        h.close()
