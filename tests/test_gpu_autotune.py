"""The autotuner on the GPU: a one-pass coordinate descent in each mode on
small graphs. tune() checks every candidate's distances against those of the
starting parameters; afterwards the tuned set is installed and its results
equal the oracle's."""
import numpy as np
import pytest

import graphgen
import oracle
from paper_2503_00430_amd import autotune
from tests.gpu_util import gpu_bfs, library, say, upload

pytestmark = pytest.mark.gpu


def quiet(*_):
    pass


@pytest.mark.parametrize("name, mode", [("rmat12", "single"), ("rmat12", "batch"), ("grid64", "graph")])
def test_tune_one_pass(name, mode):
    import torch
    bfs = library()
    g = graphgen.rmat(12) if name == "rmat12" else graphgen.grid(64)
    say("autotune", name, mode)
    gh = upload(g, bfs.BFS_SORT_NEIGHBORS)
    srcs = graphgen.sources(g, 4, seed=77)
    best = autotune.tune(gh, srcs, mode, passes=1, log=quiet)
    assert best == bfs.bfs_get_params(gh)
    space = {"single": autotune.SINGLE_SPACE, "graph": autotune.GRAPH_SPACE, "batch": autotune.BATCH_SPACE}[mode]
    defaults = bfs.bfs_default_params()
    for k, v in best.items():
        assert v in space.get(k, []) or v == defaults[k], (k, v)
    if mode == "batch":
        out = torch.empty((len(srcs), g.n), dtype=torch.uint8, device="cuda")
        bfs.bfs_run_batch(gh, np.asarray(srcs, np.int32), out)
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.msbfs_dist8(g, [int(s) for s in srcs]))
    else:
        for s in srcs:
            d, _ = gpu_bfs(gh, s, parent=False)
            np.testing.assert_array_equal(d, oracle.bfs(g, int(s), want_parent=False)[0])
    gh.close()
