"""CPU checks of the autotuner: its graph classes, the cached table of tuned
parameters, the cache lookup, and the coordinate descent on objectives
whose optimum is known."""
import json
import re

import numpy as np
import pytest

import graphgen
from paper_2503_00430_amd import autotune


def info(n, nnz, dmax):
    return {"n": n, "nnz": nnz, "max_degree": dmax}


def quiet(*_):
    pass


def test_graph_class_boundaries():
    assert autotune.graph_class(info(1 << 22, 128_302_284, 100_000)) == "n2^22_dense_hubs"
    assert autotune.graph_class(info(1 << 24, 60_714_986, 4)) == "n2^24_sparse_flat"
    # average degree nnz / n: below 7 sparse (the top-down-only class of
    # Section 3), below 24 mid, else dense
    assert autotune.graph_class(info(1024, 7 * 1024 - 1, 10)) == "n2^10_sparse_flat"
    assert autotune.graph_class(info(1024, 7 * 1024, 10)) == "n2^10_mid_flat"
    assert autotune.graph_class(info(1024, 24 * 1024 - 1, 10)) == "n2^10_mid_flat"
    assert autotune.graph_class(info(1024, 24 * 1024, 10)) == "n2^10_dense_flat"
    # hubs: a row longer than 64 times the average degree
    assert autotune.graph_class(info(1024, 8 * 1024, 8 * 64)).endswith("_flat")
    assert autotune.graph_class(info(1024, 8 * 1024, 8 * 64 + 1)).endswith("_hubs")


@pytest.mark.parametrize("make, cls", [
    (lambda: graphgen.rmat(14), "n2^14_dense_hubs"),
    (lambda: graphgen.grid(128), "n2^14_sparse_flat"),
    (lambda: graphgen.urand(1 << 14, 8), "n2^14_mid_flat"),
])
def test_graph_class_of_generated_graphs(make, cls):
    g = make()
    assert autotune.graph_class(info(g.n, g.nnz, int(np.diff(g.row_ptr).max()))) == cls


def test_cached_table_names_known_parameters_and_candidates():
    import paper_2503_00430_amd as bfs
    defaults = bfs.bfs_default_params()
    allowed = {}
    for space in (autotune.SINGLE_SPACE, autotune.GRAPH_SPACE, autotune.BATCH_SPACE):
        for k, vals in space.items():
            allowed.setdefault(k, set()).update(vals)
    table = json.load(open(autotune.DEFAULT_FILE))
    assert table
    for cls, params in table.items():
        assert re.fullmatch(r"n2\^\d+_(sparse|mid|dense)_(hubs|flat)", cls), cls
        for k, v in params.items():
            assert k in defaults, (cls, k)
            assert v in allowed[k] or v == defaults[k], (cls, k, v)


def test_load_tuned(tmp_path):
    key = info(1 << 10, 8 * 1024, 10)
    cls = autotune.graph_class(key)
    good = tmp_path / "t.json"
    good.write_text(json.dumps({cls: {"alpha": 30}, "n2^11_mid_flat": {"alpha": 8}}))
    assert autotune.load_tuned(key, str(good)) == {"alpha": 30}
    assert autotune.load_tuned(info(1 << 12, 8 * 4096, 10), str(good)) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.load_tuned(key, str(bad)) == {}
    assert autotune.load_tuned(key, str(tmp_path / "missing.json")) == {}


class Device:
    """Stands in for a graph handle: holds the installed parameters and
    counts measurements."""

    def __init__(self, objective, reject=lambda p: False):
        self.params, self.calls = {}, 0
        self.objective, self.reject = objective, reject

    def apply(self, p):
        if self.reject(p):
            return False
        self.params = dict(p)
        return True

    def score(self):
        self.calls += 1
        return self.objective(self.params)


SPACE = {"a": [1, 2, 3, 4], "b": [10, 20, 30]}


def separable(p):
    return 1000.0 - 10 * (p["a"] - 3) ** 2 - abs(p["b"] - 20)


def test_descend_finds_separable_optimum_and_stops():
    d = Device(separable)
    best, sc = autotune.descend(SPACE, {"a": 1, "b": 10, "c": 7}, d.score, d.apply, passes=5, log=quiet)
    assert best == {"a": 3, "b": 20, "c": 7}
    assert d.params == best and sc == 1000.0
    # start, then two passes of 3 + 2 trials; the second changes nothing
    assert d.calls == 1 + 5 + 5


def test_descend_skips_rejected_sets():
    d = Device(separable, reject=lambda p: p["a"] == 3)
    best, _ = autotune.descend(SPACE, {"a": 1, "b": 10}, d.score, d.apply, log=quiet)
    # a = 2 and a = 4 tie behind the rejected optimum; the first one found stays
    assert best == {"a": 2, "b": 20}
    assert d.params == best
    d = Device(separable, reject=lambda p: p["a"] == 1)
    with pytest.raises(ValueError):
        autotune.descend(SPACE, {"a": 1, "b": 10}, d.score, d.apply, log=quiet)


def test_descend_needs_more_than_one_percent():
    """Each step of a up adds 0.9 %: a = 2 is not enough over a = 1, a = 3
    is (1.8 %), and a = 4 is again under 1 % over a = 3."""
    d = Device(lambda p: 100.0 * (1 + 0.009 * (p["a"] - 1)))
    best, _ = autotune.descend(SPACE, {"a": 1, "b": 10}, d.score, d.apply, log=quiet)
    assert best == {"a": 3, "b": 10}
