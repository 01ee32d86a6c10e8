/*
 * bfs.h -- C interface of libbfs, a level-synchronous direction-optimizing
 * (hybrid top-down / bottom-up) breadth-first search for AMD Instinct
 * MI355X (gfx950).
 *
 * The operation is the one the paper states in Section 1: starting from a
 * source vertex, explore an undirected graph level by level and report, for
 * every vertex, its level (hop distance).  The graph is held in compressed
 * sparse row form (the row-offset / column-index pair of Section 2,
 * Listings 1-3).  The traversal uses the three techniques of Section 2:
 * plain (non-atomic) distance stores, switching between top-down and
 * bottom-up levels, and a bitmap of visited vertices.
 *
 * Conventions shared by every entry point
 *   - Return value: BFS_OK (0) or one of the bfs_status codes below.  On
 *     error, bfs_last_error() returns a message for the calling thread and
 *     output buffers hold unspecified contents.
 *   - Handles are opaque.  Calls on one graph handle are serialised inside
 *     the library; different handles may be used from different threads.
 *   - Vertex ids are int32 in [0, n); n < 2^31.
 *   - "device pointer" means memory on the GPU the graph was created on
 *     (hipMalloc, or a PyTorch tensor on that device); "host pointer" means
 *     ordinary process memory.
 */
#ifndef BFS_H_
#define BFS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfs_graph *bfs_graph_t;
typedef struct bfs_server *bfs_server_t;

typedef enum bfs_status {
  BFS_OK = 0,
  BFS_ERR_INVALID_ARG = 1,   /* a null handle/pointer, an id out of range, a malformed CSR */
  BFS_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed, or a budget was exceeded */
  BFS_ERR_DEVICE = 3,        /* a HIP runtime call failed */
  BFS_ERR_BUSY = 4,          /* the object still has work in flight */
  BFS_ERR_NOT_READY = 5      /* a request has not finished yet */
} bfs_status;

/* Flags of bfs_create_graph. */
#define BFS_INPUT_DEVICE 0x1u   /* row_ptr / col_idx are device pointers */
#define BFS_VALIDATE 0x2u       /* check the CSR structure before accepting it */
#define BFS_VALIDATE_SYMMETRY 0x4u /* with BFS_VALIDATE: also check v in N(u) <=> u in N(v) */
#define BFS_ROWPTR32 0x8u       /* keep row offsets as int32 on the device (needs nnz < 2^31) */
#define BFS_SORT_NEIGHBORS 0x10u /* reorder each row by descending neighbour degree (ties: ascending
                                    id) in the device copy: bottom-up scans then reach frontier
                                    vertices sooner; distances are unchanged (needs nnz < 2^31) */

/* Direction policies (bfs_params.policy). */
typedef enum bfs_policy {
  /* Section 3 classifier: top-down only when the average degree nnz/n is
   * below 7 (treated as a large-diameter graph), otherwise ALPHA_BETA. */
  BFS_POLICY_AUTO = 0,
  /* Section 2, BFS-Hybrid dagger (Beamer et al.): from top-down switch to
   * bottom-up when m_f * alpha > m_u (m_f = edges of the new frontier,
   * m_u = edges of unvisited vertices); from bottom-up switch back when
   * n_f * beta < n and the frontier shrank. */
  BFS_POLICY_ALPHA_BETA = 1,
  /* Section 2, BFS-Hybrid: bottom-up exactly when the new frontier holds at
   * least 5 % of the vertices (20 * n_f >= n). */
  BFS_POLICY_FRONTIER_5PCT = 2,
  /* top-down at every level. */
  BFS_POLICY_TD_ONLY = 3
} bfs_policy;

/* Visited test of top-down levels (bfs_params.td_visited), Section 2:
   BITMAP     - BFS-VisitedBitmap: one bit per vertex, claimed with an atomic OR;
   DIST_CAS   - BFS-Conventional: the distance itself, claimed with a
                compare-and-swap from -1 (no bitmap);
   DIST_PLAIN - BFS-NonAtomic: a plain test of the distance and a plain store
                of the (agreed) new value; racing discoverers may each append
                the vertex, so frontiers can hold duplicates (counted in the
                level statistics), and every copy is expanded at the next
                level, where its discoveries can be duplicated in turn.  The
                queues then hold n + nnz entries per set; a level that
                appends more makes bfs_run fail with BFS_ERR_OUT_OF_MEMORY
                (entries past the end are dropped, never written).  On a
                wide-front lattice the copies multiply along the shortest
                paths, so this mode is expected to fail there;
   DIST_PLAIN_CULL - the same plain test and store, and duplicates still
                enter the queue, but each appender also stores the queue
                position it wrote into a per-vertex slot (plain store, last
                writer wins) and only the copy at that position is expanded,
                so duplicate work ends after one level (an n-entry array more).
                Large-degree vertices (one entry per t2-edge chunk) are not
                culled. */
typedef enum bfs_td_visited {
  BFS_TD_VISITED_BITMAP = 0,
  BFS_TD_DIST_CAS = 1,
  BFS_TD_DIST_PLAIN = 2,
  BFS_TD_DIST_PLAIN_CULL = 3
} bfs_td_visited;

/* Level-loop drivers (bfs_params.loop). */
typedef enum bfs_loop {
  BFS_LOOP_AUTO = 0,  /* GRAPH */
  BFS_LOOP_HOST = 1,  /* host issues each level and reads the level counters back */
  BFS_LOOP_GRAPH = 2, /* replay a captured hipGraph of `graph_chunk_levels` levels
                         whose kernels test device-side direction / done flags */
  BFS_LOOP_PERSISTENT = 3, /* top-down-only runs: one cooperative launch of
                              `graph_td_blocks` workgroups runs every level,
                              levels separated by a grid barrier (hybrid
                              policies fall back to HOST) */
  BFS_LOOP_QUEUED = 4 /* the host keeps `queue_ahead` levels enqueued beyond the
                         last one the device has published; each level kernel
                         reads its direction on the device, so the device never
                         waits for the host between levels */
} bfs_loop;

/* Tunables.  bfs_default_params() fills defaults; zero fields passed to
 * bfs_set_params are replaced by the defaults. */
typedef struct bfs_params {
  int32_t policy;             /* bfs_policy */
  int32_t alpha;              /* ALPHA_BETA: default 14 */
  int32_t beta;               /* ALPHA_BETA: default 24 */
  int32_t td_wave_degree;     /* top-down: vertices with degree > this get a wavefront (default 32) */
  int32_t td_block_degree;    /* top-down: degree > this get workgroups, one per
                                 td_block_degree-edge chunk (default 2048) */
  int32_t bu_wave_degree;     /* bottom-up: unvisited vertices with degree > this are
                                 scanned by the whole wavefront (default 2048) */
  int32_t block_size;         /* threads per workgroup of the level kernels (default 512) */
  int32_t loop;               /* bfs_loop */
  int32_t graph_chunk_levels; /* GRAPH loop: levels per captured graph (default 8; 1 runs
                                 as 2, since each launch checks its level modulo
                                 the chunk length) */
  int32_t collect_timing;     /* nonzero: time each level with HIP events (HOST and QUEUED loops) */
  int32_t msbfs_block_size;   /* batched search: threads per workgroup (default 256) */
  int32_t msbfs_bu_percent;   /* batched search: a level runs bottom-up when its frontier
                                 edge count exceeds this percent of nnz (default 5) */
  int32_t graph_td_blocks;    /* GRAPH / PERSISTENT loops: size of the fixed top-down roles
                                 (default 128).  GRAPH: at most this many workgroups
                                 for the small-degree role and half as many for the
                                 medium one, each taking only as many as its queue
                                 needs; the per-chunk role takes every other workgroup
                                 of the grid.  PERSISTENT: the cooperative grid. */
  int32_t bu_blocks;          /* bottom-up: workgroups of the grid, each wavefront taking an equal
                                 share of the visited words (0 = automatic: one word per
                                 wavefront up to 1024 workgroups; at most 1024) */
  int32_t queue_ahead;        /* QUEUED loop: levels kept enqueued ahead of the device (default 2,
                                 at most 64) */
  int32_t td_visited;         /* how a top-down level tells visited vertices (paper Section 2):
                                 BFS_TD_VISITED_BITMAP (default) or, for the paper's ablation and
                                 only with the top-down-only policy, BFS_TD_DIST_CAS,
                                 BFS_TD_DIST_PLAIN or BFS_TD_DIST_PLAIN_CULL */
} bfs_params;

/* One record per executed level of the last bfs_run on a graph. */
typedef struct bfs_level_stats {
  int32_t level;          /* L: expands the vertices at distance L */
  int32_t direction;      /* 0 = top-down, 1 = bottom-up */
  int64_t frontier;       /* n_f: vertices at distance L */
  int64_t frontier_edges; /* m_f: sum of their degrees */
  int64_t unvisited_edges;/* m_u when the direction of this level was chosen */
  int64_t discovered;     /* vertices found at distance L + 1 */
  int64_t scanned;        /* bottom-up: unvisited vertices of nonzero degree examined */
  int64_t examined;       /* bottom-up: neighbours examined up to the first hit */
  float ms;               /* device time of the level's direction kernels (collect_timing,
                             host loop), else 0 */
  float pad;
} bfs_level_stats;

typedef struct bfs_run_stats {
  int32_t source;
  int32_t levels;         /* number of executed levels (max distance + 1) */
  int64_t reached;        /* vertices with dist >= 0 */
  int64_t edges;          /* undirected edges in the source's component (TEPS count) */
  double device_ms;       /* HIP-event time from initialisation to the last level */
  double host_ms;         /* wall time of the bfs_run call */
  int32_t loop;           /* bfs_loop actually used */
  int32_t policy;         /* bfs_policy actually used (AUTO resolved) */
} bfs_run_stats;

typedef struct bfs_graph_info {
  int64_t n, nnz;
  int64_t isolated;       /* vertices of degree 0 */
  int64_t max_degree;
  int64_t device_bytes;   /* device memory the handle holds (graph + scratch) */
  int32_t row_ptr_bytes;  /* 4 or 8 */
  int32_t device;         /* HIP device ordinal */
} bfs_graph_info;

/* Message describing the last error on the calling thread ("" if none).
 * The pointer stays valid until the next libbfs call on that thread. */
const char *bfs_last_error(void);

/* Fills *p with the default tunables. */
int bfs_default_params(bfs_params *p);

/*
 * bfs_create_graph: make an undirected graph resident in device memory.
 *   n, nnz   vertex count (1 <= n < 2^31) and CSR entry count (>= 0).
 *   row_ptr  n+1 int64 offsets, row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing.
 *   col_idx  nnz int32 neighbour ids in [0, n).  The CSR must be symmetric
 *            (bottom-up levels scan a vertex's own row as its in-edges);
 *            duplicate entries and self-loops are tolerated but count in nnz.
 *   flags    BFS_INPUT_DEVICE / BFS_VALIDATE / BFS_VALIDATE_SYMMETRY / BFS_ROWPTR32 /
 *            BFS_SORT_NEIGHBORS.
 *   out      receives the handle.
 * The library copies the arrays (host inputs by default) to the current HIP
 * device and owns the copies until bfs_destroy_graph; the caller may free
 * its arrays on return.  Runs use the graph's stream (the null stream unless
 * bfs_graph_set_stream is called).
 * Errors: INVALID_ARG (null pointers, n out of range, a CSR check failed),
 * OUT_OF_MEMORY, DEVICE.
 */
int bfs_create_graph(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, bfs_graph_t *out);

/* Frees the graph's device memory.  Errors: INVALID_ARG (null), BUSY (a
 * server still holds requests on it). */
int bfs_destroy_graph(bfs_graph_t g);

/* Copies the device-resident CSR back to host memory, in the row order
 * the device holds (with BFS_SORT_NEIGHBORS: each row hub-first, as the
 * bottom-up levels scan it).  row_ptr_out: n+1 int64, col_idx_out: nnz int32
 * (host pointers owned by the caller).  Errors: INVALID_ARG (null), DEVICE. */
int bfs_graph_copy_csr(bfs_graph_t g, int64_t *row_ptr_out, int32_t *col_idx_out);

/* Sets the HIP stream (a hipStream_t, passed as void*) on which runs of
 * this graph are issued.  NULL selects the null stream. */
int bfs_graph_set_stream(bfs_graph_t g, void *hip_stream);

/* Reads / replaces the graph's tunables (see bfs_params). */
int bfs_set_params(bfs_graph_t g, const bfs_params *p);
int bfs_get_params(bfs_graph_t g, bfs_params *p);
int bfs_graph_info_get(bfs_graph_t g, bfs_graph_info *info);

/*
 * bfs_run: single-source hybrid BFS (Section 2: BFS-Hybrid with the visited
 * bitmap; distances written with plain stores).  Synchronous: returns after
 * the search has finished on the graph's stream.
 *   source      id in [0, n).
 *   dist_out    device int32[n]: dist_out[v] = number of edges on a shortest
 *               source-v path, -1 if v is unreachable.
 *   parent_out  device int32[n] or NULL: parent[source] = source, parent of
 *               an unreached vertex = -1, otherwise some neighbour u with
 *               dist[u] = dist[v] - 1 (which one may vary between runs).
 * Both buffers belong to the caller.  Errors: INVALID_ARG (null graph or
 * dist_out, source out of range), DEVICE.
 */
int bfs_run(bfs_graph_t g, int32_t source, int32_t *dist_out, int32_t *parent_out);

/* Statistics of the last bfs_run on g.  `levels` (may be NULL) receives up
 * to max_levels per-level records, in level order. */
int bfs_get_run_stats(bfs_graph_t g, bfs_run_stats *st, bfs_level_stats *levels, int32_t max_levels);

/*
 * bfs_run_batch: k searches at once (1 <= k <= 64) as one multi-source BFS
 * in a single persistent launch, each vertex carrying 64-bit source sets.
 *   sources   host int32[k], ids in [0, n); repeats allowed.
 *   dist_out  device uint8[k][n], row-major: dist_out[i*n + v] = min(d, 255)
 *             where d is the distance from sources[i]; 255 also marks an
 *             unreached vertex.
 * The first call on g allocates the batch scratch, which g keeps until
 * bfs_destroy_graph (counted in device_bytes): 88 bytes per vertex (three
 * 64-bit source sets and eight 64-bit distance bit planes), about nnz/64
 * bytes of queue for long rows, and a 1 KiB control block.
 * Synchronous.  Errors: INVALID_ARG (k out of range, a source out of range,
 * null pointers), OUT_OF_MEMORY (the scratch cannot be allocated), DEVICE.
 */
int bfs_run_batch(bfs_graph_t g, const int32_t *sources, int32_t k, uint8_t *dist_out);

/*
 * bfs_run_batch_noalloc: bfs_run_batch for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).  The
 * same search, with the same arguments, errors and output, but its scratch
 * lives in a fixed array of BFS_NOALLOC_SCRATCH_BYTES that the library
 * defines on every GPU it runs on (each GPU holds it until the process
 * ends); the call itself allocates nothing.  The array holds three 64-bit
 * source sets per vertex, eight distance bit planes per vertex when k >= 16,
 * about nnz/64 bytes of queue and a 1 KiB control block, so with 16 or more
 * sources a graph of up to about 1.5 million vertices fits (about 5 million
 * with fewer); a larger one is refused with INVALID_ARG, naming the bytes it
 * would need.  Every such call on one GPU shares that GPU's array, which
 * keeps the last call's contents (the search clears what it needs): the
 * library serialises these calls within the process, and a caller must not
 * run two of them concurrently from other code paths that bypass it.
 * Synchronous.  Errors: INVALID_ARG (as bfs_run_batch, or the graph does not
 * fit the array), DEVICE.
 */
#define BFS_NOALLOC_SCRATCH_BYTES (128u << 20)
int bfs_run_batch_noalloc(bfs_graph_t g, const int32_t *sources, int32_t k, uint8_t *dist_out);

/* Request states reported by bfs_serve_poll. */
typedef enum bfs_req_state {
  BFS_REQ_QUEUED = 0,
  BFS_REQ_RUNNING = 1,
  BFS_REQ_DONE = 2,
  BFS_REQ_FAILED = 3
} bfs_req_state;

typedef struct bfs_req_stats {
  int64_t t_submit_ns;  /* steady-clock times */
  int64_t t_admit_ns;
  int64_t t_done_ns;
  int32_t levels;       /* levels the request's search ran */
  int32_t batch_lanes;  /* requests sharing its batch when it was admitted */
  int64_t edges;        /* undirected edges in the source's component */
} bfs_req_stats;

/*
 * Serving: a background thread admits single-source requests, keeps every
 * graph resident, and runs requests for the same graph together as lanes
 * of a multi-source search that new requests join at level boundaries
 * (continuous batching); batches of different graphs run concurrently on
 * separate streams.
 *   hbm_budget_bytes  upper bound on the device memory the server itself
 *                     allocates for batches in flight; requests wait until
 *                     their batch fits.
 *   max_lanes         lanes per batch, 1..64.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE.
 */
int bfs_serve_create(size_t hbm_budget_bytes, int32_t max_lanes, bfs_server_t *out);

/* Stops the server after the requests in flight have finished. */
int bfs_serve_destroy(bfs_server_t s);

/*
 * Queues one request: the single-source search of bfs_run on graph g from
 * `source`.  Never waits for the GPU.  dist_out (device int32[n]) and
 * parent_out (device int32[n] or NULL) have bfs_run's meaning and must stay
 * allocated until the request reports DONE or FAILED.  The server writes
 * them from its own streams, which are not ordered with the caller's: work
 * that still writes these buffers must have completed before the call, and
 * they hold the result once the request reports DONE.
 * Errors: INVALID_ARG; OUT_OF_MEMORY when the request alone exceeds the
 * budget.
 */
int bfs_serve_submit(bfs_server_t s, bfs_graph_t g, int32_t source, int32_t *dist_out,
                     int32_t *parent_out, uint64_t *ticket);

/* Reports a request's state and, when st is not NULL, its timings.
 * Errors: INVALID_ARG (unknown ticket). */
int bfs_serve_poll(bfs_server_t s, uint64_t ticket, int32_t *state, bfs_req_stats *st);

#ifdef __cplusplus
}
#endif

#endif /* BFS_H_ */
