"""The stored oracle digests (tests/golden/digests.json) are current: the
small workloads are recomputed here from the generators and the oracle and
must match what make_digests.py stored; the file covers every full-size
workload with the expected number of sources."""
import importlib.util
import os

import graphgen
from tests.gpu_util import golden

HERE = os.path.dirname(os.path.abspath(__file__))


def _script():
    spec = importlib.util.spec_from_file_location("make_digests", os.path.join(HERE, "golden", "make_digests.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_coverage():
    d = golden()
    for name, k in [("rmat16", 16), ("rmat24", 64), ("grid4096", 16), ("rmat22", 64)]:
        assert len(d[name]["runs"]) == k and len(d[name]["sources"]) == k, name
        assert all("dist_sha256" in r for r in d[name]["runs"])
    assert all("dist8_sha256" in r for r in d["rmat22"]["runs"])
    assert d["rmat24"]["graph"]["n"] == 1 << 24 and d["grid4096"]["graph"]["n"] == 4096 * 4096
    assert len(d["pool"]) == 12 and all(len(v["runs"]) == 4 for v in d["pool"].values())


def test_small_workloads_recomputed():
    m = _script()
    d = golden()
    assert m.workload(graphgen.rmat(16), 16, 4) == d["rmat16"]
    pool = dict(m.POOL)
    for name in ("rmat14", "grid512", "urand8"):
        assert m.workload(pool[name](), 4, 4) == d["pool"][name], name
