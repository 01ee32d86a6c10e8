"""Writes tests/golden/digests.json: the oracle's results on the full-size
workloads, as SHA-256 digests plus per-level statistics.

Only the oracle (serial FIFO BFS) and the seeded input generators are used;
nothing here runs on, or reads anything from, the GPU library.  The GPU
tests and the benchmark hash their own outputs and compare them with these
digests, so every source of every full-size workload is compared bit for
bit without running the oracle on the GPU machine.

Workloads (the generators' fixed seeds):
  rmat16     RMAT scale 16, edge factor 16, 16 sources;
  rmat24     RMAT scale 24, edge factor 16, 64 sources;
  grid4096   4096 x 4096 lattice, 10 % deletion, 1 % shortcuts, 16 sources;
  rmat22     RMAT scale 22, edge factor 16, 64 sources: int32 distances and
             the batched uint8 rows min(d, 255) (255 = unreached);
  pool       the 12 serving graphs (RMAT 14/16/18/20/22/23, lattices 512^2,
             1024^2, 2048^2 without shortcuts, uniform random 2^20 vertices
             with average degree 8/16/32), 4 sources each.

Per source: sha256 of dist as little-endian int32 (and of the uint8 row for
rmat22), the reached count, m_s (undirected edges of the component), the
number of levels and the per-level frontier sizes h and degree sums mf (as
lists up to 64 levels, as a digest of the int64 arrays beyond).

    python tests/golden/make_digests.py [--only rmat16,grid4096] [--threads 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "digests.json")
LIST_LEVELS = 64

# (name, generator call) of the serving pool, in its Zipf rank order
POOL = [("rmat14", lambda: graphgen.rmat(14)), ("rmat16", lambda: graphgen.rmat(16)),
        ("rmat18", lambda: graphgen.rmat(18)), ("rmat20", lambda: graphgen.rmat(20)),
        ("rmat22", lambda: graphgen.rmat(22)), ("grid512", lambda: graphgen.grid(512, p_shortcut=0.0)),
        ("grid1024", lambda: graphgen.grid(1024, p_shortcut=0.0)),
        ("grid2048", lambda: graphgen.grid(2048, p_shortcut=0.0)),
        ("urand8", lambda: graphgen.urand(1 << 20, 8)), ("urand16", lambda: graphgen.urand(1 << 20, 16)),
        ("urand32", lambda: graphgen.urand(1 << 20, 32)), ("rmat23", lambda: graphgen.rmat(23))]


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_digest(g) -> dict:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(g.row_ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(g.col_idx, dtype="<i4").tobytes())
    return {"n": int(g.n), "nnz": int(g.nnz), "csr_sha256": h.hexdigest()}


def run_record(g, s: int, dist8: bool = False) -> dict:
    d, _ = oracle.bfs(g, int(s), want_parent=False)
    st = oracle.level_stats(g, d)
    rec = {"source": int(s), "dist_sha256": sha(d.astype("<i4")), "reached": st["reached"],
           "m_s": st["m_s"], "levels": st["depth"]}
    h, mf = st["h"].astype("<i8"), st["mf"].astype("<i8")
    if st["depth"] <= LIST_LEVELS:
        rec["h"], rec["mf"] = h.tolist(), mf.tolist()
    else:
        rec["h_sha256"], rec["mf_sha256"] = sha(h), sha(mf)
    if dist8:
        rec["dist8_sha256"] = sha(np.where((d < 0) | (d >= 255), 255, d).astype(np.uint8))
    return rec


def workload(g, k: int, threads: int, dist8: bool = False) -> dict:
    srcs = graphgen.sources(g, k)
    with ThreadPoolExecutor(threads) as ex:  # the oracle's C call releases the GIL
        runs = list(ex.map(lambda s: run_record(g, s, dist8), srcs))
    return {"graph": graph_digest(g), "sources": [int(s) for s in srcs], "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="", help="comma-separated subset of rmat16,rmat24,grid4096,rmat22,pool")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 4)
    args = ap.parse_args()
    only = set(filter(None, args.only.split(",")))
    out = json.load(open(OUT)) if os.path.exists(OUT) and only else {}
    out["generator"] = "tests/golden/make_digests.py (oracle.bfs and graphgen only)"
    jobs = {
        "rmat16": lambda: workload(graphgen.rmat(16), 16, args.threads),
        "rmat24": lambda: workload(graphgen.rmat(24), 64, args.threads),
        "grid4096": lambda: workload(graphgen.grid(4096), 16, args.threads),
        "rmat22": lambda: workload(graphgen.rmat(22), 64, args.threads, dist8=True),
        "pool": lambda: {name: workload(mk(), 4, args.threads) for name, mk in POOL},
    }
    for name, job in jobs.items():
        if only and name not in only:
            continue
        t0 = time.time()
        out[name] = job()
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
