"""The benchmark's command line on a host without a GPU: more than one GPU
is refused with a message before anything touches a device, and the byte
model it reports against the roofline matches the oracle's."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.lstrip().startswith("{")


def test_bottom_up_byte_model_matches_oracle():
    """bench.bu_launch_bytes (applied to the device's level counts) and the
    oracle's algorithmic byte model agree on every bottom-up level of a
    hybrid search."""
    sys.path.insert(0, ROOT)
    import bench
    import graphgen
    import oracle
    g = graphgen.rmat(12)
    s = int(graphgen.sources(g, 1)[0])
    d = oracle.bfs(g, s, want_parent=False)[0]
    st = oracle.level_stats(g, d)
    dirs = oracle.replay_policy(st, oracle.POLICY_ALPHA_BETA)
    profs = {L: oracle.bottom_up_profile(g, d, L) for L, x in enumerate(dirs) if x == oracle.BU}
    assert profs, "the search has no bottom-up level"
    model = oracle.algo_bytes(st, dirs, profs, row_ptr_bytes=8, with_parent=True)
    for L, prof in profs.items():
        counts = {"scanned": prof["unvisited"], "examined": prof["examined"],
                  "discovered": int(st["h"][L + 1]) if L + 1 < len(st["h"]) else 0}
        assert bench.bu_launch_bytes(counts, g.n, 8, with_parent=True) == model["levels"][L]


def test_parity_report_counts_matching_digests():
    """bench.parity counts outputs whose SHA-256 equals the oracle's digest:
    the oracle's own distances give K/K, one changed value one less."""
    sys.path.insert(0, ROOT)
    import bench
    import graphgen
    import oracle
    g, srcs, _ = bench.make_graph("rmat16")
    outs = {int(s): oracle.bfs(g, int(s), want_parent=False)[0].astype("<i4") for s in srcs}
    assert bench.parity("rmat16", outs) == f"{len(srcs)}/{len(srcs)}"
    s0 = int(srcs[0])
    outs[s0] = outs[s0].copy()
    outs[s0][np.flatnonzero(outs[s0] > 0)[0]] += 1
    assert bench.parity("rmat16", outs) == f"{len(srcs) - 1}/{len(srcs)}"
    assert graphgen is not None


def test_cpu_baseline_pins_one_core_and_reports_host():
    sys.path.insert(0, ROOT)
    import bench
    import graphgen
    g = graphgen.rmat(10)
    before = os.sched_getaffinity(0)
    out = bench.cpu_baseline(g, graphgen.sources(g, 4), budget_s=1.0)
    assert os.sched_getaffinity(0) == before
    assert out["cores"] == 1 and out["kind"] == "oracle" and out["value"] > 0
    assert "pinned to core" in out["sample"] and out["host"]["nproc"] >= 1
