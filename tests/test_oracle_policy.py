"""Pins of the derived oracle quantities: per-level statistics, the
direction-switching rules of Section 2 (BFS-Hybrid dagger alpha/beta,
BFS-Hybrid 5 %), the Section 3 classifier, the bottom-up work profile and
the byte model -- all against hand-derived values in tests/golden/."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hand_graph():
    fx = json.load(open(os.path.join(GOLDEN, "handworked_12v.json")))
    e = np.array(fx["edges"])
    return fx, graphgen.from_edges(fx["n"], e[:, 0], e[:, 1])


def test_handworked_schedules():
    fx, g = _hand_graph()
    d, _ = oracle.bfs(g, fx["source"])
    st = oracle.level_stats(g, d)
    assert oracle.replay_policy(st, oracle.POLICY_ALPHA_BETA) == fx["schedule_alpha_beta"]
    assert oracle.replay_policy(st, oracle.POLICY_FRONTIER_5PCT) == fx["schedule_frontier_5pct"]
    assert oracle.replay_policy(st, oracle.POLICY_AUTO) == fx["schedule_auto"]
    assert oracle.replay_policy(st, oracle.POLICY_TD_ONLY) == [0] * 5


def test_handworked_bottom_up_profile():
    fx, g = _hand_graph()
    d, _ = oracle.bfs(g, fx["source"])
    for L, exp in fx["bottom_up"].items():
        assert oracle.bottom_up_profile(g, d, int(L)) == exp, L


def test_handworked_bytes():
    fx, g = _hand_graph()
    d, _ = oracle.bfs(g, fx["source"])
    st = oracle.level_stats(g, d)
    dirs = oracle.replay_policy(st, oracle.POLICY_ALPHA_BETA)
    prof = {L: oracle.bottom_up_profile(g, d, L) for L, x in enumerate(dirs) if x == oracle.BU}
    b = oracle.algo_bytes(st, dirs, prof, row_ptr_bytes=8, with_parent=True)
    assert b == fx["bytes_alpha_beta_w8_parent"]


def _graph_of(spec):
    if spec["kind"] == "path":
        return graphs.path(spec["n"])[0]
    if spec["kind"] == "star":
        return graphs.star(spec["n"])[0]
    if spec["kind"] == "broom":
        return graphs.broom(spec["k"], spec["t"])
    raise ValueError(spec)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "policy_schedules.json")))["cases"],
                         ids=lambda c: c["name"])
def test_closed_form_schedules(case):
    g = _graph_of(case["graph"])
    d, _ = oracle.bfs(g, case["source"])
    st = oracle.level_stats(g, d)
    if "schedules" in case:
        for pol, exp in case["schedules"].items():
            assert oracle.replay_policy(st, pol) == exp, pol
    else:
        for pol in ("alpha_beta", "frontier_5pct"):
            spec = case[pol]
            got = oracle.replay_policy(st, pol)
            exp = [None] * st["depth"]
            for key, val in (("td_levels", oracle.TD), ("bu_levels", oracle.BU)):
                if spec[key] is not None:
                    lo, hi = spec[key]
                    for L in range(lo, hi + 1):
                        exp[L] = val
            assert got == exp, pol


def test_level_stats_invariants_random():
    g = graphgen.rmat(12)
    s = int(graphgen.sources(g, 1)[0])
    d, _ = oracle.bfs(g, s)
    st = oracle.level_stats(g, d)
    deg = g.degree
    assert st["h"].sum() == st["reached"] == (d >= 0).sum()
    assert st["mf"].sum() == deg[d >= 0].sum() == 2 * st["m_s"]
    assert st["mu"][-1] == deg[d < 0].sum()
    # bottom-up profile: found equals the next level's size, examined is
    # between found and the full scan.
    for L in range(st["depth"]):
        p = oracle.bottom_up_profile(g, d, L)
        nxt = st["h"][L + 1] if L + 1 < st["depth"] else 0
        assert p["found"] == nxt
        assert p["found"] <= p["examined"] <= p["full"]
        assert p["unvisited"] == ((d > L) | (d < 0))[deg > 0].sum()


def test_classifier_auto():
    # average degree below 7 => top-down only; RMAT (about 28) => alpha/beta.
    g = graphgen.grid(64)
    assert g.nnz < 7 * g.n
    d, _ = oracle.bfs(g, int(graphgen.sources(g, 1)[0]))
    st = oracle.level_stats(g, d)
    assert set(oracle.replay_policy(st, "auto")) == {oracle.TD}
    r = graphgen.rmat(14)
    assert r.nnz >= 7 * r.n
    d, _ = oracle.bfs(r, int(graphgen.sources(r, 1)[0]))
    st = oracle.level_stats(r, d)
    assert oracle.replay_policy(st, "auto") == oracle.replay_policy(st, "alpha_beta")
    assert oracle.BU in oracle.replay_policy(st, "auto")


def test_summary_skip_graph_premises():
    """Premises of the GPU test of a skipped frontier summary
    (tests/graphs.summary_skip): the distances its construction implies, the
    alpha/beta schedule T T T B B at alpha 75, a level-2 expected frontier
    m_f * m_u / nnz above 4 vertices per bitmap word (where a top-down level
    stops keeping the summary) and a level-3 bottom-up frontier of at most 2
    per word (where a bottom-up level would test it)."""
    g = graphs.summary_skip()
    d = oracle.bfs(g, 0, want_parent=False)[0]
    want = np.full(g.n, -1, np.int64)
    want[0], want[1] = 0, 1
    want[2:41] = 2
    pend = 64 * (1 + np.arange(80))
    want[pend[:2]] = 2
    want[pend[2:]] = 3
    leaves = 64 * 81 + np.arange(80 * 30)
    want[leaves[:60]] = 3
    want[leaves[60:]] = 4
    assert np.array_equal(d, want)
    st = oracle.level_stats(g, d)
    words = (g.n + 63) // 64
    assert st["h"].tolist() == [1, 1, 41, 138, 2340]
    assert oracle.replay_policy(st, "alpha_beta", 75, 24) == [oracle.TD] * 3 + [oracle.BU] * 2
    assert st["mf"][2] * st["mu"][2] > 4 * words * st["nnz"]
    assert st["h"][3] <= 2 * words
