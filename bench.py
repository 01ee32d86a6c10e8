"""Benchmark: hybrid BFS GTEPS on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat24]

A step is one pass of the single-source search from each of the workload's
sources (64 for RMAT scale 24).  GTEPS per source = m_s / t_s with m_s the
undirected edges of the source's component and t_s the median wall time of
its bfs_run call over the timed steps; `value` is their harmonic mean, with
the library's default level loop (a captured hipGraph).  The graph is
resident in HBM before timing starts.  Prints one JSON line.

A second, instrumented pass repeats the timed steps with the host-driven
level loop and HIP events around every level kernel (events cannot be timed
inside a captured graph); it gives the level breakdown and the roofline.

The dominant kernel is the level kernel in its bottom-up instance
(k_level<RowT, 1>): its average duration is taken from HIP events recorded
around every bottom-up launch in the timed steps, and its algorithmic bytes
per launch from the byte model (visited, row-offset, neighbour-id, frontier
and output bytes the level must move).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS (harmonic mean, 64 sources) RMAT-24; batched vs plain; p50/p99 latency"
CREATE_FLAGS = 0x10  # BFS_SORT_NEIGHBORS: rows ordered hub-first when the graph is created
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (generator call, number of sources, row offsets int32?)
    "rmat24": ("rmat", 24, 64, False),
    "rmat22": ("rmat", 22, 64, False),
    "rmat16": ("rmat", 16, 16, True),
    "grid4096": ("grid", 4096, 16, False),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_graph(name):
    import graphgen
    kind, size, nsrc, rp32 = WORKLOADS[name]
    g = graphgen.rmat(size) if kind == "rmat" else graphgen.grid(size)
    return g, graphgen.sources(g, nsrc), rp32


def make_handle(bfs, g, rp32=False):
    """The graph as every timed section creates it: hub-first rows
    (BFS_SORT_NEIGHBORS) and the autotuned parameters of its graph class.
    Returns (handle, tuned parameters applied or None)."""
    from paper_2503_00430_amd import autotune as at
    gh = bfs.bfs_create_graph(g.row_ptr, g.col_idx, CREATE_FLAGS | (bfs.BFS_ROWPTR32 if rp32 else 0))
    return gh, at.apply_tuned(gh)


def bu_launch_bytes(lv, n, row_ptr_bytes, with_parent=True):
    """Algorithmic bytes of one bottom-up level: visited words read, row
    bounds of the scanned vertices, neighbour ids up to the first hit,
    frontier bits, next-frontier and visited words written, dist (and parent)
    of the vertices found."""
    B = 8 * ((n + 63) // 64)
    p = 4 if with_parent else 0
    return (B + row_ptr_bytes * min(n + 1, 2 * lv["scanned"]) + 4 * lv["examined"] + B + 2 * B
            + (4 + p) * lv["discovered"])


def kernel_hash():
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2503_00430_amd", "csrc", "single.hip"), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per bottom-up launch from the committed rocprofv3 counter
    summary, or None when it is absent or the kernel source has changed."""
    path = os.path.join(ROOT, "profiles", f"k_level_bu_{workload}_traffic.json")
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def host_info():
    """CPU model and core counts of the machine the CPU figures ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(g, sources, budget_s=20.0):
    """The oracle (serial C BFS with parents, one thread pinned to one core)
    on the workload's sources in order, until `budget_s` of CPU time is
    spent (every source when they fit): harmonic-mean GTEPS, m_s / t_s per
    source with t_s the oracle's own clock around initialisation plus
    traversal."""
    import oracle
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})  # this thread only; restored below
    try:
        teps, t_total = [], 0.0
        for s in sources:
            d, _, secs = oracle.bfs_timed(g, int(s), want_parent=True)
            teps.append(oracle.level_stats(g, d)["m_s"] / secs)
            t_total += secs
            if t_total > budget_s:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    hm = len(teps) / sum(1.0 / t for t in teps)
    return {"value": round(hm / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{len(teps)} of the {len(sources)} sources in order on the full graph "
                      f"(budget {budget_s:.0f} s of CPU time, {t_total:.1f} s used), serial FIFO "
                      f"BFS with parents, pinned to core {core}",
            "min_gteps": round(min(teps) / 1e9, 5), "max_gteps": round(max(teps) / 1e9, 5),
            "host": host_info()}


def golden_runs(name):
    """The oracle's per-source digests of a workload (tests/golden/digests.json,
    written from the oracle by tests/golden/make_digests.py), or None."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "digests.json")) as f:
            return json.load(f)[name]["runs"]
    except (OSError, ValueError, KeyError):
        return None


def parity(name, outputs, key="dist_sha256"):
    """Compares the SHA-256 of each output with the oracle's digest of the
    same source: "k/K" sources bit-identical (outputs: {source: array})."""
    runs = golden_runs(name)
    if runs is None:
        return "no digests"
    want = {r["source"]: r[key] for r in runs}
    ok = sum(1 for s, a in outputs.items()
             if want.get(int(s)) == hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest())
    return f"{ok}/{len(outputs)}"


OMP_KINDS = {"conventional": "BFS-Conventional (CAS on dist, top-down)",
             "nonatomic": "BFS-NonAtomic (plain dist test and store, top-down)",
             "hybrid": "BFS-Hybrid (NonAtomic body, 5 % rule)",
             "visited_bitmap": "BFS-VisitedBitmap (bitmap body, 5 % rule)",
             "hybrid_dagger": "BFS-Hybrid dagger (NonAtomic body, alpha/beta)",
             "visited_bitmap_dagger": "bitmap body, alpha/beta"}


def cpu_openmp(g, sources, budget_s=4.0, max_sources=4):
    """The paper's CPU kernels in OpenMP (cpu_context/bfs_omp.c) on the
    host's cores, with parents: harmonic-mean GTEPS over a bounded sample of
    the workload's sources, and each kernel's ratio to BFS-Conventional (the
    paper's comparison; a context figure beside the serial-oracle baseline,
    not a baseline of the GPU kernels)."""
    import cpu_context
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    edges = {}
    out = {"threads": threads, "unit": "GTEPS", "host": host_info()}
    for kind, label in OMP_KINDS.items():
        teps, t_total, entries, distinct = [], 0.0, 0, 0
        for s in sources[:max_sources]:
            d, _, secs, _, ent = cpu_context.bfs(g, int(s), kind, threads, return_entries=True)
            if int(s) not in edges:
                st = oracle.level_stats(g, d)
                edges[int(s)] = (st["m_s"], st["reached"])
            teps.append(edges[int(s)][0] / secs)
            entries += ent
            distinct += edges[int(s)][1]
            t_total += secs
            if t_total > budget_s:
                break
        out[kind] = {"kernel": label, "gteps_hm": round(len(teps) / sum(1.0 / t for t in teps) / 1e9, 4),
                     "sources": len(teps), "seconds": round(t_total, 2)}
        if kind in ("nonatomic", "hybrid"):
            # frontier entries beyond the distinct vertices (top-down levels' duplicates)
            out[kind]["duplicate_frontier_share"] = round(entries / max(distinct, 1) - 1.0, 5)
    base = out["conventional"]["gteps_hm"]
    out["ratio_to_conventional"] = {k: round(out[k]["gteps_hm"] / base, 2) for k in OMP_KINDS if base > 0}
    return out


def bench_batched(bfs, torch, reps=3, cpu=True):
    """RMAT scale 22, 64 sources: one bfs_run_batch against 64 bfs_run calls;
    every batch row and every plain result hashed against the oracle's
    digests (outside the timed calls)."""
    g, sources, _ = make_graph("rmat22")
    gh, _ = make_handle(bfs, g)
    out8 = torch.empty((len(sources), g.n), dtype=torch.uint8, device="cuda")
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    bfs.bfs_run_batch(gh, sources, out8)  # warm-up
    edges, plain, plain_out = {}, [], {}
    for rep in range(reps):
        tot = 0.0
        for s in sources:
            bfs.bfs_run(gh, int(s), dist)
            run, _ = bfs.bfs_get_run_stats(gh)
            edges[int(s)] = run["edges"]
            tot += run["host_ms"]  # the call's own wall time
            if rep == reps - 1:
                plain_out[int(s)] = dist.cpu().numpy().astype("<i4")
        plain.append(tot)
    batch = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bfs.bfs_run_batch(gh, sources, out8)
        batch.append((time.perf_counter() - t0) * 1e3)
    rows = out8.cpu().numpy()
    m = sum(edges.values())
    tb, tp = statistics.median(batch), statistics.median(plain)
    del out8
    visited = ablation(bfs, torch, gh, sources[:4])
    gh.close()
    out = {"workload": "rmat22_ef16_64src", "n": g.n, "nnz": g.nnz, "batch_ms": round(tb, 3),
           "plain_64_ms": round(tp, 3), "batch_gteps": round(m / tb / 1e6, 3),
           "plain_gteps": round(m / tp / 1e6, 3), "speedup": round(tp / tb, 3),
           "parity_batch_rows": parity("rmat22", {int(s): rows[i] for i, s in enumerate(sources)},
                                       "dist8_sha256"),
           "parity_plain": parity("rmat22", plain_out),
           "visited_test_ablation_4src_td_only": visited}
    if cpu:
        out["cpu_oracle"] = cpu_baseline(g, sources, budget_s=10.0)
    return out


def bench_small(bfs, torch, reps=20, cpu=True):
    """RMAT scale 16 (int32 row offsets), 16 sources: latency of one search
    (launch-bound, cache-resident), median over `reps` runs per source."""
    g, sources, rp32 = make_graph("rmat16")
    gh, _ = make_handle(bfs, g, rp32)
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    per, outs = {}, {}
    for s in sources:
        bfs.bfs_run(gh, int(s), dist, parent)  # warm-up
        for _ in range(reps):
            bfs.bfs_run(gh, int(s), dist, parent)
            run, _ = bfs.bfs_get_run_stats(gh)
            per.setdefault(int(s), [run["edges"], [], []])
            per[int(s)][1].append(run["host_ms"])
            per[int(s)][2].append(run["device_ms"])
        outs[int(s)] = dist.cpu().numpy().astype("<i4")
    gh.close()
    host_us = [statistics.median(t) * 1e3 for _, t, _ in per.values()]
    dev_us = [statistics.median(t) * 1e3 for _, _, t in per.values()]
    teps = [e / (statistics.median(t) / 1e3) for e, t, _ in per.values()]
    out = {"workload": "rmat16_ef16_16src_int32_rowptr", "n": g.n, "nnz": g.nnz,
           "us_per_bfs_median": round(statistics.median(host_us), 2),
           "us_per_bfs_device_median": round(statistics.median(dev_us), 2),
           "gteps_hm": round(len(teps) / sum(1.0 / t for t in teps) / 1e9, 3),
           "parity": parity("rmat16", outs)}
    if cpu:
        out["cpu_oracle"] = cpu_baseline(g, sources, budget_s=5.0)
    return out


POLICY_NAMES = {1: "alpha_beta (BFS-Hybrid dagger)", 2: "frontier_5pct (BFS-Hybrid)", 3: "td_only"}


def policy_study(bfs, torch, gh, sources, reps=2):
    """Section 2's two switching rules and the top-down-only schedule that
    Section 3's classifier picks for sparse graphs, each on the same sources
    (captured loop): harmonic-mean GTEPS and the direction schedules."""
    params = bfs.bfs_get_params(gh)
    dist = torch.empty(gh.n, dtype=torch.int32, device="cuda")
    out = {}
    for pol, name in POLICY_NAMES.items():
        bfs.bfs_set_params(gh, policy=pol, loop=bfs.BFS_LOOP_GRAPH)
        bfs.bfs_run(gh, int(sources[0]), dist)
        per, sched = {}, {}
        for _ in range(reps):
            for s in sources:
                bfs.bfs_run(gh, int(s), dist)
                run, lvs = bfs.bfs_get_run_stats(gh)
                per.setdefault(int(s), [run["edges"], []])[1].append(run["host_ms"] / 1e3)
                key = "".join("TB"[lv["direction"]] for lv in lvs)
                key = key if len(key) <= 16 else f"{key[:8]}..({len(key)} levels)"
                sched[key] = sched.get(key, 0) + 1
        teps = [e / statistics.median(t) for e, t in per.values()]
        out[name] = {"gteps_hm": round(len(teps) / sum(1.0 / t for t in teps) / 1e9, 3),
                     "schedules": dict(sorted(sched.items(), key=lambda kv: -kv[1])[:4])}
    bfs.bfs_set_params(gh, **params)
    return out


TD_VISITED = {0: "VisitedBitmap (bitmap, atomic OR)", 1: "Conventional (CAS on dist)",
              2: "NonAtomic (plain dist test and store)",
              3: "NonAtomic, duplicate copies culled at expansion"}


def ablation(bfs, torch, gh, sources, reps=1):
    """Section 2's visited tests as top-down-only searches on the same
    sources (captured loop): harmonic-mean GTEPS, and for the non-atomic
    tests the share of duplicate frontier entries they created (frontier
    entries over the bitmap run's, minus one), overall and per level for the
    first source as in the paper's Figure 1 (duplicates in % of the distinct
    frontier; for long searches a summary, with the levels whose frontier
    is under 1 % of N apart)."""
    params = bfs.bfs_get_params(gh)
    dist = torch.empty(gh.n, dtype=torch.int32, device="cuda")
    out, nf_base, per_level_base = {}, None, None
    for mode, name in TD_VISITED.items():
        bfs.bfs_set_params(gh, policy=bfs.BFS_POLICY_TD_ONLY, td_visited=mode, loop=bfs.BFS_LOOP_GRAPH)
        per, nf, first_levels = {}, 0, None
        try:
            bfs.bfs_run(gh, int(sources[0]), dist)
            for _ in range(reps):
                for s in sources:
                    bfs.bfs_run(gh, int(s), dist)
                    run, lvs = bfs.bfs_get_run_stats(gh)
                    per.setdefault(int(s), [run["edges"], []])[1].append(run["host_ms"] / 1e3)
                    nf += sum(lv["frontier"] for lv in lvs)
                    if first_levels is None:
                        first_levels = np.array([lv["frontier"] for lv in lvs], dtype=np.float64)
        except bfs.BfsError as e:  # e.g. duplicates outgrowing the queues
            out[name] = {"error": str(e)}
            continue
        # edges: the component's, from the exact (bitmap) run of each source
        if nf_base is None:
            edges = {s: e for s, (e, _) in per.items()}
            nf_base = nf
            per_level_base = first_levels
        teps = [edges[s] / statistics.median(t) for s, (_, t) in per.items()]
        out[name] = {"gteps_hm": round(len(teps) / sum(1.0 / t for t in teps) / 1e9, 3),
                     "duplicate_frontier_share": round(nf / nf_base - 1.0, 5)}
        if mode >= 2 and len(first_levels) == len(per_level_base):
            pct = 100.0 * (first_levels / per_level_base - 1.0)
            small = per_level_base < 0.01 * gh.n
            if len(pct) <= 16:
                out[name]["duplicates_pct_per_level_first_source"] = [round(float(x), 2) for x in pct]
            else:
                out[name]["duplicates_pct_first_source"] = {
                    "levels": int(len(pct)), "mean": round(float(pct.mean()), 2), "max": round(float(pct.max()), 2),
                    "mean_where_frontier_under_1pct_of_n": round(float(pct[small].mean()), 2) if small.any() else None,
                    "mean_elsewhere": round(float(pct[~small].mean()), 2) if (~small).any() else None}
    bfs.bfs_set_params(gh, **params)
    return out


LOOP_NAMES = {0: "auto (captured hipGraph loop)", 1: "host loop", 2: "captured hipGraph loop",
              3: "persistent top-down kernel", 4: "queued loop"}


def bench_mesh(bfs, torch, reps=2, cpu=True):
    """4096 x 4096 perturbed lattice, 16 sources (top-down only, with the
    level loop its tuned parameters select), and the captured loop on 4 of
    the sources beside it."""
    g, sources, _ = make_graph("grid4096")
    gh, _ = make_handle(bfs, g)
    tuned_loop = bfs.bfs_get_params(gh)["loop"]
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    bfs.bfs_run(gh, int(sources[0]), dist)  # warm-up (captures the level loop)
    per, outs = {}, {}
    levels = []
    for rep in range(reps):
        for s in sources:
            bfs.bfs_run(gh, int(s), dist)
            run, _ = bfs.bfs_get_run_stats(gh)
            per.setdefault(int(s), [run["edges"], []])[1].append(run["host_ms"] / 1e3)
            levels.append(run["levels"])
            if rep == reps - 1:
                outs[int(s)] = dist.cpu().numpy().astype("<i4")
    teps = [e / statistics.median(t) for e, t in per.values()]
    captured = None
    if tuned_loop not in (0, bfs.BFS_LOOP_GRAPH):
        params = bfs.bfs_get_params(gh)
        bfs.bfs_set_params(gh, loop=bfs.BFS_LOOP_GRAPH)
        bfs.bfs_run(gh, int(sources[0]), dist)
        ct = []
        for s in sources[:4]:
            bfs.bfs_run(gh, int(s), dist)
            run, _ = bfs.bfs_get_run_stats(gh)
            ct.append(run["edges"] / (run["host_ms"] / 1e3))
        captured = round(len(ct) / sum(1.0 / t for t in ct) / 1e9, 4)
        bfs.bfs_set_params(gh, **params)
    policies = policy_study(bfs, torch, gh, sources[:4], reps=1)
    visited = ablation(bfs, torch, gh, sources[:4])
    gh.close()
    hm = len(teps) / sum(1.0 / t for t in teps) / 1e9
    mean_ms = statistics.mean(statistics.median(t) for _, t in per.values()) * 1e3
    out = {"workload": "grid4096_p0.1_16src", "n": g.n, "nnz": g.nnz, "gteps_hm": round(hm, 4),
           "loop": LOOP_NAMES.get(tuned_loop, tuned_loop), "captured_loop_gteps_hm_4src": captured,
           "ms_per_bfs": round(mean_ms, 3), "levels_mean": round(statistics.mean(levels), 1),
           "us_per_level": round(mean_ms * 1e3 / statistics.mean(levels), 2),
           "parity": parity("grid4096", outs),
           "policy_study_4src": policies, "visited_test_ablation_4src": visited}
    if cpu:
        out["cpu_oracle"] = cpu_baseline(g, sources, budget_s=10.0)
    return out


# Serving pool: RMAT scales 14-22 and 23, perturbed lattices without
# shortcuts, and uniform random graphs of 2^20 vertices; graphs are drawn
# Zipf(1.1) in this order, sources uniformly among non-isolated vertices.
SERVE_POOL = [("rmat", 14), ("rmat", 16), ("rmat", 18), ("rmat", 20), ("rmat", 22),
              ("grid", 512), ("grid", 1024), ("grid", 2048),
              ("urand", 8), ("urand", 16), ("urand", 32), ("rmat", 23)]


def _serve_graph(kind, size):
    import graphgen
    if kind == "rmat":
        return graphgen.rmat(size)
    if kind == "grid":
        return graphgen.grid(size, p_shortcut=0.0)
    return graphgen.urand(1 << 20, size)


def _component_edges(g):
    """Undirected edges of each vertex's component (TEPS numerator per source)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    a = csr_matrix((np.ones(g.nnz, np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(a, directed=False)
    per = np.bincount(lab, weights=np.diff(g.row_ptr), minlength=lab.max() + 1) / 2
    return per[lab]


SERVE_CLASSES = {"rmat": "power-law (RMAT 14-23)", "grid": "lattice (512^2-2048^2)", "urand": "uniform random (2^20)"}


def _pcts(lat_s):
    return {"p50_ms": round(float(np.percentile(lat_s, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat_s, 99)) * 1e3, 3)}


def bench_serving(bfs, torch, requests=2000, plain_fracs=(0.25, 0.5, 0.9), sat_fracs=(0.5, 0.9),
                  budget=1 << 30, seed=6000):
    """Poisson arrivals over the 12-graph pool through the server, against
    the same trace served first-come-first-served by plain bfs_run.

    One trace of `requests` requests (graph Zipf(1.1), source uniform among
    non-isolated vertices) is replayed at each rate: fractions of the plain
    FCFS capacity C (the trace's requests per second of summed bfs_run
    times, each request timed alone) and of the server's saturation rate S
    (every request submitted at once).  At every rate the server is run for
    real; the plain FCFS latencies are computed from the same requests'
    measured bfs_run times (a single queue in arrival order), and at 0.9 C
    the plain FCFS is also run for real (the host issues bfs_run at each
    arrival).  The server's memory budget (`budget`, scratch of the batches
    in flight; the graphs themselves are resident outside it) is smaller
    than the pool's batches together, so admission waits for memory."""
    graphs, handles, edges, nz, cls = [], [], [], [], []
    for kind, size in SERVE_POOL:
        g = _serve_graph(kind, size)
        graphs.append(g)
        handles.append(make_handle(bfs, g)[0])
        edges.append(_component_edges(g))
        nz.append(np.flatnonzero(g.degree > 0))
        cls.append(kind)
    rng = np.random.default_rng(seed)
    zipf = 1.0 / np.arange(1, len(graphs) + 1) ** 1.1
    zipf /= zipf.sum()
    gid = rng.choice(len(graphs), size=requests, p=zipf)
    src = [int(nz[k][rng.integers(len(nz[k]))]) for k in gid]
    gaps = rng.exponential(1.0, size=requests)  # unit-rate Poisson gaps, scaled per rate
    m_s = np.array([edges[k][s] for k, s in zip(gid, src)])
    req_cls = np.array([cls[k] for k in gid])
    # output buffers: a pool per graph, reused once a request is done
    pool_size = 128
    bufs = [[torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(pool_size)] for g in graphs]
    torch.cuda.synchronize()

    # each request alone through bfs_run (the plain path's service times)
    dist = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
    for k in range(len(graphs)):
        bfs.bfs_run(handles[k], int(nz[k][0]), dist[k])
    run_s = np.empty(requests)
    for i, (k, s) in enumerate(zip(gid, src)):
        bfs.bfs_run(handles[k], s, dist[k])
        run_s[i] = bfs.bfs_get_run_stats(handles[k])[0]["host_ms"] / 1e3
    plain_rate = requests / run_s.sum()

    def serve(arrivals):
        srv = bfs.bfs_serve_create(budget, 64)
        free = [list(range(pool_size)) for _ in graphs]
        inflight = {}
        lat = np.zeros(requests)
        wait = np.zeros(requests)
        i = 0
        t0_ns = time.perf_counter_ns()  # CLOCK_MONOTONIC, as the server's timestamps
        t0 = t0_ns / 1e9
        while i < requests or inflight:
            now = time.perf_counter() - t0
            while i < requests and arrivals[i] <= now and free[gid[i]]:
                b = free[gid[i]].pop()
                t = bfs.bfs_serve_submit(srv, handles[gid[i]], src[i], bufs[gid[i]][b])
                inflight[t] = (i, b)
                i += 1
            for t in list(inflight):
                state, st = bfs.bfs_serve_poll(srv, t)
                if state == bfs.BFS_REQ_DONE:
                    j, b = inflight.pop(t)
                    # latency from the request's arrival time in the trace
                    lat[j] = (st["t_done_ns"] - t0_ns) / 1e9 - arrivals[j]
                    wait[j] = (st["t_admit_ns"] - st["t_submit_ns"]) / 1e9
                    free[gid[j]].append(b)
                elif state == bfs.BFS_REQ_FAILED:
                    raise RuntimeError("a served request failed")
            if i < requests and not inflight and arrivals[i] > now:
                time.sleep(min(arrivals[i] - now, 0.001))
        wall = time.perf_counter() - t0
        bfs.bfs_serve_destroy(srv)
        return lat, wall, wait

    def plain_model(arrivals):
        finish, fl = 0.0, np.empty(requests)
        for j in range(requests):
            finish = max(finish, arrivals[j]) + run_s[j]
            fl[j] = finish - arrivals[j]
        return fl, max(finish, arrivals[-1])

    def plain_real(arrivals):
        fl = np.empty(requests)
        t0 = time.perf_counter()
        for j in range(requests):
            now = time.perf_counter() - t0
            if arrivals[j] > now:
                time.sleep(arrivals[j] - now)
            bfs.bfs_run(handles[gid[j]], src[j], dist[gid[j]])
            fl[j] = time.perf_counter() - t0 - arrivals[j]
        return fl, time.perf_counter() - t0

    def per_class(lat):
        return {c: _pcts(lat[req_cls == c]) for c in SERVE_CLASSES if (req_cls == c).any()}

    # saturation: every request submitted at once
    lat0, wall0, _ = serve(np.zeros(requests))
    sat = requests / wall0
    out = {"pool": [f"{k}{z}" for k, z in SERVE_POOL], "requests_per_rate": requests,
           "budget_bytes": budget, "classes": SERVE_CLASSES,
           "requests_per_class": {c: int((req_cls == c).sum()) for c in SERVE_CLASSES},
           "saturation_rps": round(sat, 1), "plain_fcfs_capacity_rps": round(plain_rate, 1),
           "saturation_gteps": round(m_s.sum() / wall0 / 1e9, 3),
           "alone_ms_per_class": {c: _pcts(run_s[req_cls == c]) for c in SERVE_CLASSES},
           "rates": []}
    for base, fracs, name in ((plain_rate, plain_fracs, "plain_capacity"), (sat, sat_fracs, "saturation")):
        for frac in fracs:
            rate = frac * base
            arrivals = np.cumsum(gaps) / rate
            lat, wall, wait = serve(arrivals)
            fl, fwall = plain_model(arrivals)
            row = {"rate_rps": round(rate, 1), "of": f"{frac} x {name}", **_pcts(lat),
                   "p99_ms_per_class": per_class(lat),
                   "admission_wait_p99_ms": round(float(np.percentile(wait, 99)) * 1e3, 3),
                   "gteps": round(m_s.sum() / wall / 1e9, 3),
                   "plain_fcfs_model": {**_pcts(fl), "p99_ms_per_class": per_class(fl),
                                        "gteps": round(m_s.sum() / fwall / 1e9, 3)}}
            if name == "plain_capacity" and frac == max(fracs):
                rl, rwall = plain_real(arrivals)
                row["plain_fcfs_run"] = {**_pcts(rl), "p99_ms_per_class": per_class(rl),
                                         "gteps": round(m_s.sum() / rwall / 1e9, 3)}
            out["rates"].append(row)
            log(f"serving {row['of']}: {row['rate_rps']} rps p50 {row['p50_ms']} p99 {row['p99_ms']} ms")
    for h in handles:
        h.close()
    return out


def copy_bandwidth(torch, reps=10):
    """A plain 1 GiB device-to-device copy timed with events on the current
    stream: (bytes read + bytes written) / time, in GB/s (the streaming
    ceiling this GPU reaches, beside the published 8 TB/s)."""
    x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    e1.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    torch.cuda.empty_cache()
    return round(2 * (1 << 30) / secs / 1e9, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, mesh and serving sections")
    ap.add_argument("--levels-json", default=None,
                    help="write the instrumented pass's per-level records of every search to this file "
                         "(the last --steps passes over the sources, in launch order)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving section (12-graph pool)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched section (RMAT-22, 64 sources), e.g. to profile its kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the search runs on a single device).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        # A copy of known size: 1 GiB read and 1 GiB written per launch.
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "launches": 5}))
        return
    import paper_2503_00430_amd as bfs
    if not os.path.exists(bfs.library_path()):
        from paper_2503_00430_amd import build as libbuild
        libbuild.build()
    global autotune
    from paper_2503_00430_amd import autotune
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.serving_only:
        print(json.dumps({"serving": bench_serving(bfs, torch)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": bench_batched(bfs, torch, cpu=False)}), flush=True)
        return

    t0 = time.time()
    g, sources, rp32 = make_graph(args.workload)
    log(f"generated {args.workload}: n={g.n} nnz={g.nnz} in {time.time() - t0:.1f} s")
    gh, tuned = make_handle(bfs, g, rp32)
    info = bfs.bfs_graph_info_get(gh)
    params = bfs.bfs_get_params(gh)
    # one output pair per source (HBM has room: 2 x 64 x 4N bytes at scale
    # 24), so every timed search's own result can be hashed afterwards
    dists = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in sources]
    parents = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in sources]

    def step(record):
        for i, s in enumerate(sources):
            bfs.bfs_run(gh, int(s), dists[i], parents[i])
            if record is not None:
                run, levels = bfs.bfs_get_run_stats(gh)
                record.append((int(s), run, levels))

    # headline pass: the library's default level loop (captured hipGraph)
    for _ in range(args.warmup):
        step(None)
    log("warmup done")
    records = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(records)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    log(f"timed {args.steps} steps in {t_end - t_start:.3f} s")
    # the distances of the last timed step, against the oracle's digests
    timed_parity = parity(args.workload, {int(s): dists[i].cpu().numpy().astype("<i4")
                                          for i, s in enumerate(sources)})
    log(f"parity of the timed results: {timed_parity}")

    # per-source median wall time -> TEPS; harmonic mean over sources
    def hm_gteps(recs, key):
        per = {}
        for s, run, _ in recs:
            per.setdefault(s, {"edges": run["edges"], "t": []})["t"].append(run[key] / 1e3)
        teps = [v["edges"] / statistics.median(v["t"]) for v in per.values()]
        return len(teps) / sum(1.0 / t for t in teps) / 1e9

    gteps_hm = hm_gteps(records, "host_ms")
    gteps_dev_hm = hm_gteps(records, "device_ms")

    # instrumented pass: the host-driven loop records HIP events around every
    # level kernel on the launch stream (captured graphs cannot carry timed
    # events); the same kernels run, so it gives the level breakdown and the
    # bottom-up kernel's roofline
    bfs.bfs_set_params(gh, loop=bfs.BFS_LOOP_HOST, collect_timing=1)
    step(None)
    inst = []
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step(inst)
    torch.cuda.synchronize()
    gteps_host_loop = hm_gteps(inst, "host_ms")
    if args.levels_json:
        with open(args.levels_json, "w") as f:
            json.dump([{"source": s, "run": run, "levels": lvs} for s, run, lvs in inst], f)
    bfs.bfs_set_params(gh, **params)
    policies = None if args.no_extras else policy_study(bfs, torch, gh, sources[:16])

    # level breakdown and the bottom-up kernel's roofline
    runs = len(inst)
    td_ms = sum(lv["ms"] for _, _, lvs in inst for lv in lvs if lv["direction"] == 0) / runs
    bu_levels = [lv for _, _, lvs in inst for lv in lvs if lv["direction"] == 1]
    bu_ms = sum(lv["ms"] for lv in bu_levels) / runs
    roofline = None
    if bu_levels:
        avg_s = statistics.mean(lv["ms"] for lv in bu_levels) / 1e3
        avg_bytes = statistics.mean(bu_launch_bytes(lv, g.n, info["row_ptr_bytes"]) for lv in bu_levels)
        achieved = avg_bytes / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(args.workload),
                    "kernel": "k_level<long, 1> (bottom-up instance)",
                    "avg_launch_us": round(avg_s * 1e6, 2),
                    "algo_bytes_per_launch": int(avg_bytes), "launches": len(bu_levels),
                    "measured_in": "instrumented host-loop pass over the same sources and steps "
                                   "(HIP events around every level kernel)"}
    # per-level profile of the first source (stderr, for reading)
    s0, run0, lvs0 = inst[0]
    log(f"source {s0}: {run0['levels']} levels, host {run0['host_ms']:.3f} ms, "
        f"device {run0['device_ms']:.3f} ms")
    for lv in lvs0:
        log(f"  L{lv['level']:<3d} {'TB'[lv['direction']]} n_f={lv['frontier']:<9d} "
            f"m_f={lv['frontier_edges']:<10d} found={lv['discovered']:<9d} "
            f"scanned={lv['scanned']:<9d} examined={lv['examined']:<10d} {lv['ms'] * 1e3:9.1f} us")
    schedules = {}
    for _, _, lvs in records[: len(sources)]:
        key = "".join("TB"[lv["direction"]] for lv in lvs)
        schedules[key] = schedules.get(key, 0) + 1

    out = {
        "metric": METRIC,
        "value": round(gteps_hm, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t_end - t_start) * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_plain_hybrid_bfs", "n": g.n, "nnz": g.nnz,
                   "sources": len(sources), "row_ptr_bytes": info["row_ptr_bytes"],
                   "policy": "auto (alpha/beta for average degree >= 7, else top-down only)",
                   "neighbour_order": "hub-first (BFS_SORT_NEIGHBORS, at graph creation)",
                   "loop": "captured hipGraph level loop (library default)",
                   "params": {k: v for k, v in bfs.bfs_get_params(gh).items()
                              if k not in ("collect_timing",)},
                   "tuned_params_applied": bool(tuned), "parents": True},
        "parity": {"dist_bit_exact_vs_oracle": timed_parity,
                   "how": "SHA-256 of each timed search's distances against the oracle's digest "
                          "of the same source (tests/golden/digests.json)"},
        "roofline": roofline,
        "gteps_device_time_hm": round(gteps_dev_hm, 3),
        "gteps_host_loop_hm": round(gteps_host_loop, 3),
        "td_ms_per_bfs": round(td_ms, 4),
        "bu_ms_per_bfs": round(bu_ms, 4),
        "direction_schedules": schedules,
        "policy_study_16src": policies,
    }
    gh.close()
    del dists, parents
    torch.cuda.empty_cache()
    if roofline is not None:
        roofline["measured_copy_GBps"] = copy_bandwidth(torch)
    cpu = not args.no_cpu_baseline
    if not args.no_extras:
        log("small section (rmat16 latency)")
        out["small"] = bench_small(bfs, torch, cpu=cpu)
        log("batched section (rmat22)")
        out["batched"] = bench_batched(bfs, torch, cpu=cpu)
        torch.cuda.empty_cache()
        log("mesh section (grid4096)")
        out["mesh"] = bench_mesh(bfs, torch, cpu=cpu)
        torch.cuda.empty_cache()
        log("serving section (12-graph pool)")
        out["serving"] = bench_serving(bfs, torch)
        torch.cuda.empty_cache()
    if cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(g, sources)
        log("cpu context (OpenMP kernels of the paper)")
        out["cpu_openmp_context"] = cpu_openmp(g, sources)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
