"""Checks of the synthetic input generators (shape, determinism, CSR form).
These are properties of inputs, not parity checks."""
import hashlib

import numpy as np
import pytest

import graphgen


def _check_csr(g):
    rp, col = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == len(col) == g.nnz
    assert (np.diff(rp) >= 0).all()
    assert ((col >= 0) & (col < g.n)).all()
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert (rows != col).all(), "self-loop"
    # sorted, unique rows
    key = rows.astype(np.int64) * g.n + col
    assert (np.diff(key) > 0).all()
    # symmetric
    rkey = col.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(rkey), key)


def _digest(g):
    h = hashlib.sha256()
    h.update(g.row_ptr.tobytes()); h.update(g.col_idx.tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("mk", [lambda: graphgen.rmat(12), lambda: graphgen.grid(40),
                                lambda: graphgen.urand(5000, 8)], ids=["rmat", "grid", "urand"])
def test_csr_form_and_determinism(mk):
    g1, g2 = mk(), mk()
    _check_csr(g1)
    assert _digest(g1) == _digest(g2)


def test_from_edges_matches_numpy():
    rng = np.random.default_rng(0)
    n = 300
    u = rng.integers(0, n, 2000); v = rng.integers(0, n, 2000)
    g = graphgen.from_edges(n, u, v)
    _check_csr(g)
    keep = u != v
    pairs = set()
    for a, b in zip(u[keep], v[keep]):
        pairs.add((int(a), int(b))); pairs.add((int(b), int(a)))
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    assert set(zip(rows.tolist(), g.col_idx.tolist())) == pairs


def test_rmat_shape():
    g = graphgen.rmat(14)
    assert g.n == 1 << 14
    deg = g.degree
    # heavy tail and many isolated vertices are characteristic of R-MAT
    assert deg.max() > 50 * deg.mean()
    assert 0.05 < (deg == 0).mean() < 0.6
    assert g.nnz <= 2 * 16 * g.n


def test_rmat_thread_independent():
    import subprocess, sys, os
    code = ("import graphgen,hashlib;g=graphgen.rmat(11);h=hashlib.sha256();"
            "h.update(g.row_ptr.tobytes());h.update(g.col_idx.tobytes());print(h.hexdigest())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = set()
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=root)
        outs.add(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                text=True, check=True).stdout.strip())
    assert len(outs) == 1


def test_grid_shape():
    w = 64
    g = graphgen.grid(w)
    n = w * w
    lattice = 2 * w * (w - 1)
    und = g.nnz // 2
    # about 90 % of lattice edges plus up to 1 % shortcuts
    assert 0.85 * lattice < und < 0.95 * lattice + 0.01 * n
    g0 = graphgen.grid(w, p_delete=0.0, p_shortcut=0.0)
    assert g0.nnz == 2 * lattice


def test_grid_shortcut_radius():
    w = 50
    g = graphgen.grid(w, p_delete=0.0, p_shortcut=0.05, radius=3)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    r1, c1 = divmod(rows, w); r2, c2 = divmod(g.col_idx.astype(np.int64), w)
    md = np.abs(r1 - r2) + np.abs(c1 - c2)
    assert md.max() <= 3 and md.min() >= 1
    assert (md > 1).sum() > 0


def test_urand_degree():
    g = graphgen.urand(1 << 14, 16)
    assert abs(g.nnz / g.n - 16) < 0.5


def test_sources_distinct_nonisolated():
    g = graphgen.rmat(12)
    s = graphgen.sources(g, 64)
    assert len(s) == 64 and len(set(s.tolist())) == 64
    assert (g.degree[s] > 0).all()
    assert np.array_equal(s, graphgen.sources(g, 64))
    small = graphgen.from_edges(6, [0, 1], [1, 2])
    assert sorted(graphgen.sources(small, 10).tolist()) == [0, 1, 2]
