"""GPU parity of the batched multi-source search (bfs_run_batch): every row
of the uint8 [k][N] output must equal min(oracle distance, 255), with 255
for unreached vertices."""
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


def run_batch(bfs, gh, sources):
    import torch
    out = torch.empty((len(sources), gh.n), dtype=torch.uint8, device="cuda")
    bfs.bfs_run_batch(gh, np.asarray(sources, np.int32), out)
    return out.cpu().numpy()


def expect(g, sources):
    return oracle.msbfs_dist8(g, [int(s) for s in sources])


@pytest.fixture(scope="module")
def rmat16():
    return graphgen.rmat(16)


@pytest.mark.parametrize("k", [1, 2, 63, 64])
def test_rmat16_batches(bfs, rmat16, k):
    g = rmat16
    say("batch rmat16 k", k)
    gh = upload(g)
    srcs = graphgen.sources(g, k, seed=900 + k)
    got = run_batch(bfs, gh, srcs)
    np.testing.assert_array_equal(got, expect(g, srcs))
    gh.close()


@pytest.mark.parametrize("pct", [0, 1, 5, 30, 100])
def test_direction_thresholds(bfs, rmat16, pct):
    g = rmat16
    say("batch rmat16 bu_percent", pct)
    gh = upload(g, bfs.BFS_ROWPTR32)
    bfs.bfs_set_params(gh, msbfs_bu_percent=pct)
    srcs = graphgen.sources(g, 64, seed=31)
    np.testing.assert_array_equal(run_batch(bfs, gh, srcs), expect(g, srcs))
    gh.close()


def test_duplicates_isolated_and_components(bfs):
    say("batch duplicates / isolated / components")
    g = graphgen.from_edges(200, np.concatenate([np.arange(99), 100 + np.arange(80)]),
                            np.concatenate([np.arange(1, 100), 101 + np.arange(80)]))
    gh = upload(g)
    srcs = [0, 0, 50, 199, 150, 99, 100, 180, 50]  # repeats; 199 isolated
    np.testing.assert_array_equal(run_batch(bfs, gh, srcs), expect(g, srcs))
    gh.close()


def test_saturation_long_path(bfs):
    say("batch path 700 saturation")
    g, _ = graphs.path(700)
    gh = upload(g)
    srcs = [0, 699, 350, 10]
    got = run_batch(bfs, gh, srcs)
    np.testing.assert_array_equal(got, expect(g, srcs))
    assert got[0, 254] == 254 and got[0, 255] == 255 and got[0, 699] == 255
    gh.close()


@pytest.mark.parametrize("n", [15, 16, 17, 40, 700])
def test_bit_planes_on_paths(bfs, n):
    """Batches of 16 or more searches keep their distances as bit planes
    and write the rows after the last level: paths whose largest distance
    needs 4 planes, exactly 5, more, and the saturated 255."""
    say("batch bit planes path", n)
    g, _ = graphs.path(n)
    gh = upload(g)
    srcs = ([0, n - 1] * 8 + list(range(0, n, max(1, n // 8))))[:24]
    for k in (15, 16, len(srcs)):
        np.testing.assert_array_equal(run_batch(bfs, gh, srcs[:k]), expect(g, srcs[:k]))
    gh.close()


def test_bit_planes_repeats_isolated_hubs(bfs):
    say("batch bit planes: repeats, isolated, hub rows")
    g = graphgen.from_edges(200, np.concatenate([np.arange(99), 100 + np.arange(80)]),
                            np.concatenate([np.arange(1, 100), 101 + np.arange(80)]))
    gh = upload(g)
    srcs = [0, 0, 50, 199, 150, 99, 100, 180, 50] * 3  # repeats; 199 isolated
    np.testing.assert_array_equal(run_batch(bfs, gh, srcs), expect(g, srcs))
    gh.close()
    k = 20000
    u = np.concatenate([np.zeros(k, np.int64), np.arange(1, 300), [5000] * 3000])
    v = np.concatenate([np.arange(1, k + 1), np.arange(2, 301), np.arange(10000, 13000)])
    g = graphgen.from_edges(k + 1, u, v)
    gh = upload(g)
    srcs = [0, 1, 150, 5000, 12000, k, 7, 299, 300, 301, 9999, 10000, 10001, 13000, 13001, 42, 0]
    for pct in (0, 100):
        bfs.bfs_set_params(gh, msbfs_bu_percent=pct)
        np.testing.assert_array_equal(run_batch(bfs, gh, srcs), expect(g, srcs))
    gh.close()


def test_closed_forms(bfs):
    for name, mk in sorted(graphs.CLOSED_FORMS.items()):
        g, f = mk()
        say("batch closed form", name)
        gh = upload(g)
        srcs = [0] if name == "binary_tree" else list(range(0, g.n, max(1, g.n // 20)))[:64]
        got = run_batch(bfs, gh, srcs)
        for i, s in enumerate(srcs):
            d = f(s)
            np.testing.assert_array_equal(got[i], np.where((d < 0) | (d >= 255), 255, d))
        gh.close()


def test_hub_rows(bfs):
    """Rows far longer than a wavefront, in both directions."""
    say("batch hub rows")
    k = 20000
    u = np.concatenate([np.zeros(k, np.int64), np.arange(1, 300), [5000] * 3000])
    v = np.concatenate([np.arange(1, k + 1), np.arange(2, 301), np.arange(10000, 13000)])
    g = graphgen.from_edges(k + 1, u, v)
    gh = upload(g)
    for pct in (0, 100):
        bfs.bfs_set_params(gh, msbfs_bu_percent=pct)
        srcs = [0, 1, 150, 5000, 12000, k]
        np.testing.assert_array_equal(run_batch(bfs, gh, srcs), expect(g, srcs))
    gh.close()


def test_bad_arguments(bfs, rmat16):
    import torch
    gh = upload(rmat16)
    out = torch.empty((65, gh.n), dtype=torch.uint8, device="cuda")
    with pytest.raises(bfs.BfsError):
        bfs.bfs_run_batch(gh, np.arange(65, dtype=np.int32), out)
    out1 = torch.empty((1, gh.n), dtype=torch.uint8, device="cuda")
    with pytest.raises(bfs.BfsError):
        bfs.bfs_run_batch(gh, np.array([gh.n], np.int32), out1)
    gh.close()


@pytest.mark.parametrize("config", ["bench", "default"])
def test_rmat22_config(bfs, config):
    """RMAT scale 22, 64 sources in one launch, in the benchmark's
    configuration (hub-first rows, tuned parameters) and with defaults: every
    row equals the oracle's min(d, 255) (SHA-256 digests written from the
    oracle), and so does every one of the 64 plain searches the benchmark
    times beside the batch."""
    import bench
    from tests.gpu_util import check_graph_digest, golden, sha256
    rec = golden()["rmat22"]
    say("generating rmat22")
    g, srcs, _ = bench.make_graph("rmat22")
    check_graph_digest(g, rec["graph"])
    assert [int(s) for s in srcs] == rec["sources"]
    gh = bench.make_handle(bfs, g)[0] if config == "bench" else upload(g)
    say("batch rmat22 k=64", config, bfs.bfs_get_params(gh))
    got = run_batch(bfs, gh, srcs)
    for i, r in enumerate(rec["runs"]):
        assert sha256(got[i]) == r["dist8_sha256"], f"row {i} (source {r['source']}) differs"
    if config == "bench":
        import torch
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for r in rec["runs"]:
            bfs.bfs_run(gh, r["source"], dist)
            assert sha256(dist.cpu().numpy().astype("<i4")) == r["dist_sha256"], r["source"]
    gh.close()
