// C interface of libbfs: error reporting, tunables, graph residency.
//
// bfs_create_graph makes the CSR of an undirected graph resident in device
// memory (the row-offset / column-index arrays of the paper's Listings 1-3)
// together with the per-graph scratch the searches reuse: visited and
// frontier bitmaps (Section 2, BFS-VisitedBitmap), frontier queues split by
// degree class, and the device control block.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.h"

namespace bfsmi {

namespace {
thread_local std::string t_error;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_error = buf;
  return code;
}

void clear_error() { t_error.clear(); }

int resolved_policy(const bfs_graph *g) {
  int p = g->params.policy;
  if (p == BFS_POLICY_AUTO) p = (g->nnz < 7 * g->n) ? BFS_POLICY_TD_ONLY : BFS_POLICY_ALPHA_BETA;
  return p;
}

static void free_dev(void *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <class T>
static hipError_t dev_alloc(T *&p, size_t count, int64_t &acct) {
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e == hipSuccess) {
    p = static_cast<T *>(q);
    acct += (int64_t)bytes;
  }
  return e;
}

// Queue capacities.  With a test-and-set visited check (bitmap or
// compare-and-swap) every vertex enters the frontier once, so a set's small
// and medium queues hold at most n entries; every large vertex has degree
// > t2, so there are at most nnz / t2 of them, holding at most
// nnz / t2 + count chunks of t2 edges.  The visited test of plain loads and
// stores (Section 2, BFS-NonAtomic) lets racing discoverers append a vertex
// again, up to once per examined edge, so its queues are sized for the
// edges as well; a level that still outgrows them is stopped and reported.
static int64_t queue_capacity(const bfs_graph *g) {
  int64_t cap = g->n;
  if (g->params.td_visited >= BFS_TD_DIST_PLAIN) cap += g->nnz;
  return std::min<int64_t>(cap, INT32_MAX);
}

static int64_t large_capacity(const bfs_graph *g) {
  int64_t t2 = std::max<int64_t>(g->params.td_block_degree, 1);
  int64_t cap = 2 * (g->nnz / t2) + 2;
  if (g->params.td_visited >= BFS_TD_DIST_PLAIN) cap *= 8;
  return std::min<int64_t>(cap, INT32_MAX);
}

template <class T>
static int grow_queues(bfs_graph *g, T *(&q)[2], int64_t &have, int64_t cap, const char *what) {
  if (cap <= have) return BFS_OK;
  for (int s = 0; s < 2; ++s) {
    if (q[s]) {
      g->device_bytes -= have * (int64_t)sizeof(T);
      void *p = q[s];
      free_dev(p);
      q[s] = nullptr;
    }
  }
  have = 0;
  for (int s = 0; s < 2; ++s) {
    if (dev_alloc(q[s], cap, g->device_bytes) != hipSuccess) {
      if (s == 1) {  // keep the pair consistent: release the first of the two
        g->device_bytes -= cap * (int64_t)sizeof(T);
        void *p = q[0];
        free_dev(p);
        q[0] = nullptr;
      }
      return fail(BFS_ERR_OUT_OF_MEMORY, "cannot allocate %lld %s queue entries", (long long)cap, what);
    }
  }
  have = cap;
  return BFS_OK;
}

int alloc_single_scratch(bfs_graph *g) {
  const int64_t qcap = queue_capacity(g);
  int64_t small_have = g->q_cap, medium_have = g->q_cap;
  int rc = grow_queues(g, g->qs, small_have, qcap, "small-vertex");
  if (!rc) rc = grow_queues(g, g->qm, medium_have, qcap, "medium-vertex");
  // both kinds now hold at least the smaller of the two counts
  g->q_cap = std::min(small_have, medium_have);
  if (rc) return rc;
  rc = grow_queues(g, g->ql, g->ql_cap, large_capacity(g), "large-vertex");
  if (rc) return rc;
  if (g->params.td_visited == BFS_TD_DIST_PLAIN_CULL && !g->slot &&
      dev_alloc(g->slot, g->n, g->device_bytes) != hipSuccess)
    return fail(BFS_ERR_OUT_OF_MEMORY, "cannot allocate the %lld-entry queue-slot array", (long long)g->n);
  return BFS_OK;
}

void release_graph_exec(bfs_graph *g) {
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->gexec = nullptr;
  g->graph = nullptr;
  g->gexec_levels = 0;
}

static void destroy(bfs_graph *g) {
  DeviceGuard dg(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  release_graph_exec(g);
  void *ptrs[] = {g->rp, g->col, g->iso, g->head, g->headc, g->nb4, g->hrank, g->rpc, g->vis, g->bm[0], g->bm[1], g->sm[0], g->sm[1], g->qs[0], g->qs[1],
                  g->qm[0], g->qm[1], g->ql[0], g->ql[1], g->slot, g->ctl, g->recs, g->partials,
                  g->ms.seen, g->ms.front, g->ms.next, g->ms.counters, g->ms.hq, g->ms.planes};
  for (void *p : ptrs) free_dev(p);
  if (g->ctl_host) (void)hipHostFree(g->ctl_host);
  if (g->ev_start) (void)hipEventDestroy(g->ev_start);
  if (g->ev_stop) (void)hipEventDestroy(g->ev_stop);
  for (hipEvent_t e : g->level_events) (void)hipEventDestroy(e);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  delete g;
}

static int validate_csr(int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                        bool symmetry) {
  if (rp[0] != 0) return fail(BFS_ERR_INVALID_ARG, "row_ptr[0] = %lld, expected 0", (long long)rp[0]);
  if (rp[n] != nnz)
    return fail(BFS_ERR_INVALID_ARG, "row_ptr[n] = %lld, expected nnz = %lld", (long long)rp[n],
                (long long)nnz);
  for (int64_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v])
      return fail(BFS_ERR_INVALID_ARG, "row_ptr decreases at vertex %lld", (long long)v);
  for (int64_t j = 0; j < nnz; ++j)
    if (col[j] < 0 || col[j] >= n)
      return fail(BFS_ERR_INVALID_ARG, "col_idx[%lld] = %d out of range", (long long)j, col[j]);
  if (symmetry) {
    std::vector<int32_t> sorted(col, col + nnz);
    for (int64_t v = 0; v < n; ++v) std::sort(sorted.begin() + rp[v], sorted.begin() + rp[v + 1]);
    for (int64_t u = 0; u < n; ++u)
      for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t v = col[j];
        if (!std::binary_search(sorted.begin() + rp[v], sorted.begin() + rp[v + 1], (int32_t)u))
          return fail(BFS_ERR_INVALID_ARG, "CSR not symmetric: edge %lld->%d has no reverse",
                      (long long)u, v);
      }
  }
  return BFS_OK;
}

static bfs_params default_params() {
  bfs_params p;
  std::memset(&p, 0, sizeof(p));
  p.policy = BFS_POLICY_AUTO;
  p.alpha = 14;
  p.beta = 24;
  p.td_wave_degree = 32;
  p.td_block_degree = 2048;
  p.bu_wave_degree = 2048;
  p.block_size = 512;
  p.loop = BFS_LOOP_AUTO;
  p.graph_chunk_levels = 8;
  p.collect_timing = 0;
  p.msbfs_block_size = 256;
  p.msbfs_bu_percent = 5;
  p.graph_td_blocks = 128;
  p.queue_ahead = 2;
  p.td_visited = BFS_TD_VISITED_BITMAP;
  return p;
}

static int check_params(const bfs_params &p) {
  if (p.policy < BFS_POLICY_AUTO || p.policy > BFS_POLICY_TD_ONLY)
    return fail(BFS_ERR_INVALID_ARG, "unknown policy %d", p.policy);
  if (p.alpha < 1 || p.beta < 1) return fail(BFS_ERR_INVALID_ARG, "alpha and beta must be >= 1");
  if (p.td_wave_degree < 1 || p.td_block_degree < 64 || p.td_block_degree <= p.td_wave_degree)
    return fail(BFS_ERR_INVALID_ARG,
                "need 1 <= td_wave_degree < td_block_degree and td_block_degree >= 64");
  if (p.bu_wave_degree < 1) return fail(BFS_ERR_INVALID_ARG, "bu_wave_degree must be >= 1");
  for (int bs : {p.block_size, p.msbfs_block_size})
    if (bs < 64 || bs > 1024 || bs % 64)
      return fail(BFS_ERR_INVALID_ARG, "block sizes must be multiples of 64 in [64, 1024]");
  if (p.loop < BFS_LOOP_AUTO || p.loop > BFS_LOOP_QUEUED)
    return fail(BFS_ERR_INVALID_ARG, "unknown loop driver %d", p.loop);
  if (p.graph_chunk_levels < 1 || p.graph_chunk_levels > 4096)
    return fail(BFS_ERR_INVALID_ARG, "graph_chunk_levels must be in [1, 4096]");
  if (p.graph_td_blocks < 1 || p.graph_td_blocks > 512)
    return fail(BFS_ERR_INVALID_ARG, "graph_td_blocks must be in [1, 512]");
  if (p.td_visited < BFS_TD_VISITED_BITMAP || p.td_visited > BFS_TD_DIST_PLAIN_CULL)
    return fail(BFS_ERR_INVALID_ARG, "unknown td_visited %d", p.td_visited);
  if (p.queue_ahead < 1 || p.queue_ahead > 64)
    return fail(BFS_ERR_INVALID_ARG, "queue_ahead must be in [1, 64]");
  if (p.bu_blocks < 0 || p.bu_blocks > kMaxBlocks)
    return fail(BFS_ERR_INVALID_ARG, "bu_blocks must be in [0, %d]", kMaxBlocks);
  if (p.msbfs_bu_percent < 0 || p.msbfs_bu_percent > 100)
    return fail(BFS_ERR_INVALID_ARG, "msbfs_bu_percent must be in [0, 100]");
  return BFS_OK;
}

}  // namespace bfsmi

using namespace bfsmi;

extern "C" {

const char *bfs_last_error(void) { return bfsmi::t_error.c_str(); }

int bfs_default_params(bfs_params *p) {
  clear_error();
  if (!p) return fail(BFS_ERR_INVALID_ARG, "null params");
  *p = default_params();
  return BFS_OK;
}

int bfs_create_graph(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                     uint32_t flags, bfs_graph_t *out) {
  clear_error();
  if (!out) return fail(BFS_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (n < 1 || n >= ((int64_t)1 << 31))
    return fail(BFS_ERR_INVALID_ARG, "n = %lld outside [1, 2^31)", (long long)n);
  if (nnz < 0) return fail(BFS_ERR_INVALID_ARG, "nnz < 0");
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(BFS_ERR_INVALID_ARG, "null CSR array");
  if (flags & ~(BFS_INPUT_DEVICE | BFS_VALIDATE | BFS_VALIDATE_SYMMETRY | BFS_ROWPTR32 |
                BFS_SORT_NEIGHBORS))
    return fail(BFS_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  const bool rp32 = flags & BFS_ROWPTR32;
  if (rp32 && nnz >= ((int64_t)1 << 31))
    return fail(BFS_ERR_INVALID_ARG, "BFS_ROWPTR32 needs nnz < 2^31");

  int dev = 0;
  BFS_HIP(hipGetDevice(&dev));

  // Host view of the CSR (device inputs are copied back for the checks and
  // the degree statistics).
  std::vector<int64_t> rp_copy;
  std::vector<int32_t> col_copy;
  const int64_t *rp = row_ptr;
  const int32_t *col = col_idx;
  if (flags & BFS_INPUT_DEVICE) {
    rp_copy.resize(n + 1);
    BFS_HIP(hipMemcpy(rp_copy.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    rp = rp_copy.data();
    if ((flags & BFS_VALIDATE) && nnz > 0) {
      col_copy.resize(nnz);
      BFS_HIP(hipMemcpy(col_copy.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
      col = col_copy.data();
    }
  }
  if (flags & BFS_VALIDATE) {
    int rc = validate_csr(n, nnz, rp, col, flags & BFS_VALIDATE_SYMMETRY);
    if (rc) return rc;
  } else if (rp[n] != nnz) {
    return fail(BFS_ERR_INVALID_ARG, "row_ptr[n] = %lld, expected nnz = %lld", (long long)rp[n],
                (long long)nnz);
  }

  bfs_graph *g = new (std::nothrow) bfs_graph;
  if (!g) return fail(BFS_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->device = dev;
  g->n = n;
  g->nnz = nnz;
  g->words = (n + 63) / 64;
  g->rp64 = !rp32;
  g->params = default_params();

  // Degree statistics and the isolated-vertex bitmap (degree-0 vertices and
  // the ids past n in the last word are marked, so searches treat them as
  // visited from the start).
  std::vector<uint64_t> iso(g->words, 0);
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rp[v + 1] - rp[v];
    if (d == 0) {
      iso[v >> 6] |= 1ull << (v & 63);
      ++g->isolated;
    }
    g->max_degree = std::max(g->max_degree, d);
  }
  for (int64_t v = n; v < g->words * 64; ++v) iso[v >> 6] |= 1ull << (v & 63);
  // per-word ranks into the compacted head records of non-isolated vertices
  std::vector<uint32_t> hrank(g->words);
  {
    uint64_t r = 0;
    for (int64_t w = 0; w < g->words; ++w) {
      hrank[w] = (uint32_t)r;
      r += (uint64_t)__builtin_popcountll(~iso[w]);
    }
  }
  if (g->max_degree > INT32_MAX) {
    delete g;
    return fail(BFS_ERR_INVALID_ARG, "a row has more than 2^31 - 1 entries");
  }

  auto bail = [&](int code) {
    destroy(g);
    return code;
  };
  int64_t &acct = g->device_bytes;
  hipError_t e = hipSuccess;
#define ALLOC(ptr, count)                                                                   \
  do {                                                                                      \
    e = dev_alloc(ptr, count, acct);                                                        \
    if (e != hipSuccess)                                                                    \
      return bail(fail(BFS_ERR_OUT_OF_MEMORY, "device allocation of %s failed: %s", #ptr,   \
                       hipGetErrorString(e)));                                              \
  } while (0)
  if (rp32) {
    int32_t *p = nullptr;
    ALLOC(p, n + 1);
    g->rp = p;
  } else {
    int64_t *p = nullptr;
    ALLOC(p, n + 1);
    g->rp = p;
  }
  ALLOC(g->col, nnz);
  ALLOC(g->iso, g->words);
  ALLOC(g->head, n);
  ALLOC(g->headc, std::max<int64_t>(1, n - g->isolated));
  if (g->max_degree <= 4) ALLOC(g->nb4, n);
  if (nnz < ((int64_t)1 << 32)) ALLOC(g->rpc, std::max<int64_t>(1, n - g->isolated));
  ALLOC(g->hrank, g->words);
  ALLOC(g->vis, g->words);
  ALLOC(g->bm[0], g->words);
  ALLOC(g->bm[1], g->words);
  for (int sh = 0; sh <= kSumMaxShift; ++sh) {
    const int64_t bits = (g->words + ((int64_t)1 << sh) - 1) >> sh;
    if (bits <= kSumMaxBits) {
      g->sshift = sh;
      g->swords = (bits + 63) / 64;
      break;
    }
  }
  if (g->sshift >= 0) {
    ALLOC(g->sm[0], g->swords);
    ALLOC(g->sm[1], g->swords);
  }
  ALLOC(g->ctl, 1);
  ALLOC(g->partials, kPartialsAlloc);
  g->rec_cap = 1 << 16;
  ALLOC(g->recs, g->rec_cap);
#undef ALLOC
  {
    int rc = alloc_single_scratch(g);
    if (rc) return bail(rc);
  }
  e = hipHostMalloc((void **)&g->ctl_host, sizeof(Ctl), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return bail(fail(BFS_ERR_OUT_OF_MEMORY, "pinned allocation failed"));
  std::memset(g->ctl_host, 0, sizeof(Ctl));
  e = hipHostGetDevicePointer((void **)&g->ctl_host_dev, g->ctl_host, 0);
  if (e != hipSuccess) return bail(fail(BFS_ERR_DEVICE, "hipHostGetDevicePointer failed"));

  // Copies.
  const hipMemcpyKind kind = (flags & BFS_INPUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (rp32) {
    std::vector<int32_t> r32(n + 1);
    for (int64_t v = 0; v <= n; ++v) r32[v] = (int32_t)rp[v];
    e = hipMemcpy(g->rp, r32.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice);
  } else {
    e = hipMemcpy(g->rp, rp, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && nnz > 0) e = hipMemcpy(g->col, col_idx, sizeof(int32_t) * nnz, kind);
  if (e == hipSuccess) e = hipMemcpy(g->iso, iso.data(), sizeof(uint64_t) * g->words, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->hrank, hrank.data(), sizeof(uint32_t) * g->words, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(g->ctl, 0, sizeof(Ctl));
  if (e == hipSuccess) e = hipMemset(g->partials, 0, sizeof(unsigned long long) * kPartialsAlloc);
  if (e == hipSuccess) e = hipEventCreate(&g->ev_start);
  if (e == hipSuccess) e = hipEventCreate(&g->ev_stop);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess)
    return bail(fail(BFS_ERR_DEVICE, "graph upload failed: %s", hipGetErrorString(e)));
  {
    int rc = build_head(g);
    if (!rc && (flags & BFS_SORT_NEIGHBORS)) rc = sort_neighbors_by_degree(g, rp);
    if (rc) return bail(rc);
  }
  *out = g;
  return BFS_OK;
}

int bfs_destroy_graph(bfs_graph_t g) {
  clear_error();
  if (!g) return fail(BFS_ERR_INVALID_ARG, "null graph");
  {
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->server_refs.load() != 0)
      return fail(BFS_ERR_BUSY, "graph still has %d requests in a server", g->server_refs.load());
  }
  destroy(g);
  return BFS_OK;
}

int bfs_graph_copy_csr(bfs_graph_t g, int64_t *row_ptr_out, int32_t *col_idx_out) {
  clear_error();
  if (!g || !row_ptr_out || (g->nnz > 0 && !col_idx_out)) return fail(BFS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  DeviceGuard dg(g->device);
  if (g->rp64) {
    BFS_HIP(hipMemcpy(row_ptr_out, g->rp, sizeof(int64_t) * (g->n + 1), hipMemcpyDeviceToHost));
  } else {
    std::vector<int32_t> r32(g->n + 1);
    BFS_HIP(hipMemcpy(r32.data(), g->rp, sizeof(int32_t) * (g->n + 1), hipMemcpyDeviceToHost));
    for (int64_t v = 0; v <= g->n; ++v) row_ptr_out[v] = r32[v];
  }
  if (g->nnz > 0) BFS_HIP(hipMemcpy(col_idx_out, g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost));
  return BFS_OK;
}

int bfs_graph_set_stream(bfs_graph_t g, void *hip_stream) {
  clear_error();
  if (!g) return fail(BFS_ERR_INVALID_ARG, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  g->stream = static_cast<hipStream_t>(hip_stream);
  return BFS_OK;
}

int bfs_set_params(bfs_graph_t g, const bfs_params *p) {
  clear_error();
  if (!g || !p) return fail(BFS_ERR_INVALID_ARG, "null argument");
  bfs_params q = *p;
  const bfs_params d = default_params();
#define DEF(f) \
  if (q.f == 0) q.f = d.f
  DEF(alpha); DEF(beta); DEF(td_wave_degree); DEF(td_block_degree); DEF(bu_wave_degree);
  DEF(block_size); DEF(graph_chunk_levels); DEF(msbfs_block_size); DEF(graph_td_blocks);
  DEF(queue_ahead);
#undef DEF
  int rc = check_params(q);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g->mu);
  DeviceGuard dg(g->device);
  g->params = q;
  release_graph_exec(g);
  return alloc_single_scratch(g);
}

int bfs_get_params(bfs_graph_t g, bfs_params *p) {
  clear_error();
  if (!g || !p) return fail(BFS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  *p = g->params;
  return BFS_OK;
}

int bfs_graph_info_get(bfs_graph_t g, bfs_graph_info *info) {
  clear_error();
  if (!g || !info) return fail(BFS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g->mu);
  info->n = g->n;
  info->nnz = g->nnz;
  info->isolated = g->isolated;
  info->max_degree = g->max_degree;
  info->device_bytes = g->device_bytes + g->ms.bytes;
  info->row_ptr_bytes = g->rp64 ? 8 : 4;
  info->device = g->device;
  return BFS_OK;
}

int bfs_run(bfs_graph_t g, int32_t source, int32_t *dist_out, int32_t *parent_out) {
  clear_error();
  if (!g) return fail(BFS_ERR_INVALID_ARG, "null graph");
  if (!dist_out) return fail(BFS_ERR_INVALID_ARG, "null dist_out");
  if (source < 0 || source >= g->n)
    return fail(BFS_ERR_INVALID_ARG, "source %d outside [0, %lld)", source, (long long)g->n);
  std::lock_guard<std::mutex> lk(g->mu);
  DeviceGuard dg(g->device);
  return run_single(g, source, dist_out, parent_out);
}

int bfs_get_run_stats(bfs_graph_t g, bfs_run_stats *st, bfs_level_stats *levels, int32_t max_levels) {
  clear_error();
  if (!g || !st) return fail(BFS_ERR_INVALID_ARG, "null argument");
  if (levels && max_levels < 0) return fail(BFS_ERR_INVALID_ARG, "max_levels < 0");
  std::lock_guard<std::mutex> lk(g->mu);
  *st = g->last;
  if (levels) {
    int32_t m = std::min<int32_t>(max_levels, (int32_t)g->last_levels.size());
    std::copy(g->last_levels.begin(), g->last_levels.begin() + m, levels);
  }
  return BFS_OK;
}

int bfs_run_batch(bfs_graph_t g, const int32_t *sources, int32_t k, uint8_t *dist_out) {
  clear_error();
  if (!g) return fail(BFS_ERR_INVALID_ARG, "null graph");
  if (!sources || !dist_out) return fail(BFS_ERR_INVALID_ARG, "null argument");
  if (k < 1 || k > 64) return fail(BFS_ERR_INVALID_ARG, "k = %d outside [1, 64]", k);
  for (int i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(BFS_ERR_INVALID_ARG, "sources[%d] = %d outside [0, %lld)", i, sources[i],
                  (long long)g->n);
  std::lock_guard<std::mutex> lk(g->mu);
  DeviceGuard dg(g->device);
  return run_batch(g, sources, k, dist_out, nullptr);
}

int bfs_run_batch_noalloc(bfs_graph_t g, const int32_t *sources, int32_t k, uint8_t *dist_out) {
  clear_error();
  if (!g) return fail(BFS_ERR_INVALID_ARG, "null graph");
  if (!sources || !dist_out) return fail(BFS_ERR_INVALID_ARG, "null argument");
  if (k < 1 || k > 64) return fail(BFS_ERR_INVALID_ARG, "k = %d outside [1, 64]", k);
  for (int i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(BFS_ERR_INVALID_ARG, "sources[%d] = %d outside [0, %lld)", i, sources[i],
                  (long long)g->n);
  std::lock_guard<std::mutex> lk(g->mu);
  DeviceGuard dg(g->device);
  return run_batch_static(g, sources, k, dist_out);
}

}  // extern "C"
