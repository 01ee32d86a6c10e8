// Internal declarations of libbfs (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bfs.h"

namespace bfsmi {

constexpr int kWave = 64;

enum Dir : int32_t { kTD = 0, kBU = 1 };
// How the frontier of the level about to run is held: as queues (the usual
// top-down form) or, right after a switch back from bottom-up, as the bitmap
// the bottom-up level wrote.
enum Conv : int32_t { kConvNone = 0, kConvB2Q = 2 };
enum Bucket : int32_t { kSmall = 0, kMedium = 1, kLarge = 2 };
enum Publish : int32_t { kPubEvery = 0, kPubFinal = 1 };

// Per-level record written on the device by the decide step.
struct LevelRec {
  int32_t level, dir;
  int64_t n_f, m_f, m_u, found, scanned, examined;
};

// Device-resident control block of one single-source search.  The level
// state is written only by the decide step (and by the init kernel); the
// level kernels add only to the queue counts.  Every kernel reads what it
// needs from here, so a captured sequence of kernels stays valid from level
// to level.
struct alignas(256) Ctl {
  int32_t level;   // level about to run: expands vertices at distance `level`
  int32_t dir;     // its direction (kTD / kBU)
  int32_t done;    // nonzero once a level found nothing
  int32_t qcur;    // queue set holding the current frontier
  int32_t bcur;    // bitmap holding the current frontier
  int32_t conv;    // kConvB2Q: a top-down `level` reads its frontier from the bitmap
  int32_t policy;  // resolved bfs_policy (never AUTO)
  int32_t alpha, beta;
  int32_t rec_cap;  // capacity of the LevelRec array
  int32_t levels_done;
  int32_t overflow; // nonzero: a level appended more entries than a queue holds
                    // (entries past the end were dropped; the search stops)
  int32_t classless; // DevG::classless of this search
  int32_t sum_ok[2];  // nonzero: summary s has a bit for every word of bitmap s
                      // that holds a frontier vertex (bottom-up levels may test it)
  int64_t n;        // vertex count
  int64_t nnz;      // adjacency entries (twice the undirected edges)
  int64_t n_f;      // size of the current frontier
  int64_t m_f;      // sum of degrees over the current frontier
  int64_t m_u;      // sum of degrees over vertices not yet visited
  int64_t sum_mf;   // sum of m_f over all levels so far (= 2 * TEPS edge count)
  int64_t reached;  // vertices visited so far
  unsigned int qcnt[2][3];  // entries held by queue set s, bucket b (large: one per vertex)
  unsigned int qchunk[2];   // td_block_degree-edge chunks of the large vertices of set s
  unsigned int qcap[2];     // capacity of each small/medium queue, of each large queue
  int32_t *dist;    // outputs of the current search
  int32_t *parent;
  Ctl *mirror;      // host-mapped copy the decide step publishes after every level
  uint32_t bar_count;  // grid barrier of the persistent top-down kernel
  uint32_t bar_gen;
  uint32_t seq;     // publications so far (the mirror's copy is written last)
  int32_t pub_mode; // kPubEvery: publish after every level; kPubFinal: only the last
  uint32_t seq_wip; // the mirror's copy: number of the publication being written
                    // (written first, so a reader can tell a torn copy)
};

// Level kernels run at most kMaxBlocks workgroups; each writes its counts
// (found, degree sum of found, scanned, examined) to its own slot of the
// partials array, which the decide step reduces and clears.  No two
// workgroups add to the same device word.
constexpr int kMaxBlocks = 1024;
constexpr int kPartials = 4;
// The fused decide step's accumulators (kArriveGroups x kPartials) and
// arrival counters (one per group and one over the groups) follow the
// partials in the same allocation, each in its own 128-byte line.
constexpr int kArriveGroups = 8;
constexpr int kLineU64 = 16;
constexpr size_t kAccOffset = (size_t)kMaxBlocks * kPartials;
constexpr size_t kArriveOffset = kAccOffset + (size_t)kArriveGroups * kPartials * kLineU64;
constexpr size_t kPartialsAlloc = kArriveOffset + (size_t)(kArriveGroups + 1) * kLineU64;

// Occupancy summaries of the frontier bitmaps: at most this many bits
// (32 KB, copied into each bottom-up workgroup's LDS), and at most 8 bitmap
// words per bit (a bottom-up wavefront stores whole summary bytes).
constexpr int64_t kSumMaxBits = (int64_t)1 << 18;
constexpr int kSumMaxShift = 3;

// Everything a single-source kernel needs, passed by value.
template <class RowT>
struct DevG {
  const RowT *rp;
  const int32_t *col;
  const uint64_t *iso;  // bit set: vertex has degree 0, or id >= n (tail of last word)
  const int4 *head;     // per vertex: {degree, first three neighbours or -1}
  const int4 *headc;    // the same records for the non-isolated vertices only, in id order
  const int4 *nb4;      // graphs of maximum degree <= 4: per vertex all four neighbours
                        // (-1 past the row's end), else null
  const uint32_t *hrank;  // per word: non-isolated vertices in the words before it
  const uint32_t *rpc;  // row offsets of the non-isolated vertices in headc order (null
                        // when nnz >= 2^32: then rp is read)
  uint64_t *vis;        // visited bitmap
  uint64_t *bm[2];      // frontier bitmaps (current / next alternate)
  uint64_t *sm[2];      // their occupancy summaries: bit i set if words [i << sshift,
                        // (i + 1) << sshift) of bm[b] may hold a set bit (a superset)
  int32_t sshift;       // log2 of the bitmap words per summary bit (-1: no summaries)
  int32_t swords;       // 64-bit words per summary
  int32_t *qs[2];       // queue sets: small-degree vertices
  int32_t *qm[2];       //             medium-degree vertices
  uint64_t *ql[2];      //             large-degree vertices, one entry per chunk: chunk << 32 | v
  Ctl *ctl;
  LevelRec *recs;
  unsigned long long *partials;  // [kMaxBlocks][kPartials], then accumulators and arrivals
  int64_t n;
  int64_t words;        // 64-bit words per bitmap
  int32_t t1, t2, tbu;  // degree thresholds (td_wave_degree, td_block_degree, bu_wave_degree)
  int32_t td_visited;   // bfs_td_visited of the top-down claims
  uint32_t qcap, lcap;  // entries each small/medium queue and each large queue holds
  int32_t *slot;        // BFS_TD_DIST_PLAIN_CULL only (else null): per vertex, the
                        // queue position its last appender wrote
  int32_t classless;    // top-down only, every degree <= t1: discoveries all go to the
                        // small queue without reading their degree, and a level's
                        // frontier degree sum m_f is added up when it is expanded
  int32_t pers;         // nonzero inside the persistent kernel: data that workgroups of
                        // one level hand to the next (queues, slots, plainly tested
                        // distances) goes through the device-coherent level of the
                        // memory system instead of an XCD's cache
};

// Scratch of the batched (multi-source) search, allocated on first use.
struct MsScratch {
  uint64_t *seen = nullptr, *front = nullptr, *next = nullptr;
  unsigned long long *counters = nullptr;
  uint64_t *hq = nullptr;  // chunk queue of long top-down rows
  int64_t hq_cap = 0;
  uint64_t *planes = nullptr;  // 8 bit planes of the distances, [8][n]
  int64_t words = 0;
  size_t bytes = 0;
};

}  // namespace bfsmi

struct bfs_graph {
  int device = 0;
  int64_t n = 0, nnz = 0, words = 0;
  bool rp64 = true;
  void *rp = nullptr;
  int32_t *col = nullptr;
  uint64_t *iso = nullptr;
  int4 *head = nullptr;  // {degree, first three neighbours or -1} per vertex
  int4 *headc = nullptr;  // head records of the non-isolated vertices only, in id order
  int4 *nb4 = nullptr;    // maximum degree <= 4: all four neighbours per vertex (-1 past the end)
  uint32_t *hrank = nullptr;  // per word: count of non-isolated vertices in earlier words
  uint32_t *rpc = nullptr;  // row offsets in headc order (allocated when nnz < 2^32)
  uint64_t *vis = nullptr;
  uint64_t *bm[2] = {nullptr, nullptr};
  uint64_t *sm[2] = {nullptr, nullptr};  // occupancy summaries of bm (see DevG)
  int32_t sshift = -1;
  int64_t swords = 0;
  int32_t *qs[2] = {nullptr, nullptr};
  int32_t *qm[2] = {nullptr, nullptr};
  uint64_t *ql[2] = {nullptr, nullptr};
  int64_t ql_cap = 0;
  int64_t q_cap = 0;  // entries of each small/medium queue
  int32_t *slot = nullptr;  // n entries, allocated for BFS_TD_DIST_PLAIN_CULL
  bfsmi::Ctl *ctl = nullptr;
  bfsmi::Ctl *ctl_host = nullptr;  // pinned, coherent, device-mapped mirror of ctl
  bfsmi::Ctl *ctl_host_dev = nullptr;  // its device-side address
  uint32_t pub_seq = 0;  // last publication number (continues across runs)
  unsigned long long *partials = nullptr;
  bfsmi::LevelRec *recs = nullptr;
  int32_t rec_cap = 0;
  int64_t isolated = 0, max_degree = 0;
  int64_t device_bytes = 0;
  hipStream_t stream = nullptr;      // caller's stream (null stream by default)
  hipStream_t cap_stream = nullptr;  // private stream used for graph capture
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  std::vector<hipEvent_t> level_events;
  bfs_params params{};
  std::mutex mu;
  std::atomic<int> server_refs{0};
  // last run
  bfs_run_stats last{};
  std::vector<bfs_level_stats> last_levels;
  // captured level loop
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int gexec_levels = 0;
  // batched search
  bfsmi::MsScratch ms;
};

namespace bfsmi {

// Error reporting (thread-local message; returns `code`).
int fail(int code, const char *fmt, ...);
void clear_error();

// Sets the graph's device current for the lifetime of the guard.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

int resolved_policy(const bfs_graph *g);
int build_head(bfs_graph *g);  // fills g->head from the resident CSR
// BFS_SORT_NEIGHBORS (reorder.hip); host_rp: a host copy of the row offsets
int sort_neighbors_by_degree(bfs_graph *g, const int64_t *host_rp);
int alloc_single_scratch(bfs_graph *g);  // (re)allocates the large-vertex queues
void release_graph_exec(bfs_graph *g);

// Single-source search (single.hip).
int run_single(bfs_graph *g, int32_t source, int32_t *dist, int32_t *parent);

// Batched search (msbfs.hip).  `stream` overrides the graph's stream when
// not null.  Writes k rows of uint8 distances.
int run_batch(bfs_graph *g, const int32_t *sources, int32_t k, uint8_t *dist8, hipStream_t stream);
// The same search with its scratch in the library's fixed per-device array
// (bfs_run_batch_noalloc): allocates nothing.
int run_batch_static(bfs_graph *g, const int32_t *sources, int32_t k, uint8_t *dist8);

}  // namespace bfsmi

#define BFS_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::bfsmi::fail(BFS_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
