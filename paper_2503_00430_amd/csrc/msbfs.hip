// Batched multi-source BFS: up to 64 searches share one traversal.
//
// Every vertex carries three 64-bit sets, bit i standing for search i:
//   seen[v]  - searches that have reached v,
//   front[v] - searches for which v is on the current frontier,
//   next[v]  - candidate bits gathered during the running level.
// A level is the level-synchronous step of the single-source search
// (Section 2, Listing 1) applied to all searches at once:
//   top-down  - each vertex with front[v] != 0 pushes front[v] & ~seen[n]
//               into next[n] of every neighbour n (atomicOr on the word);
//   bottom-up - each vertex with unfinished searches ORs the front sets of
//               its neighbours, stopping as soon as every search it still
//               lacks has been found (the early exit of Section 2,
//               BFS-Hybrid, extended to 64 searches);
// then a finalize pass turns next into the new frontier and marks it seen.
// The direction of each level follows the frontier's edge count.
//
// Distances.  A small batch writes each level into the uint8 distance rows
// as it is found.  Those stores fill 64-byte row segments only in part, one
// per search and level, so a batch of kMsPlaneMinK or more searches instead
// keeps the distances as 8 bit planes per vertex (bit i of plane b is bit b
// of search i's distance) and writes the rows once, in whole segments, after
// the last level.
//
// The whole search is one cooperative launch: levels are separated by
// grid-wide barriers.  Each workgroup adds its level totals into device
// accumulators with atomics; after one barrier every workgroup reads them
// and takes the same decision on the next direction and on termination.

#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>

#include "common.h"
#include "device_util.h"

namespace cg = cooperative_groups;

namespace bfsmi {
namespace {

// Device control block of one batched search.
// Every workgroup takes the same per-level decision from the level's totals,
// so none is published here; the totals of level L are accumulated into
// acc[L % 3] (one 128-byte line each), and level L's decide clears
// acc[(L + 2) % 3], whose last readers passed a grid barrier before and whose
// next writers come after another.  hcnt[L & 1] counts the chunk entries of
// level L's frontier (queued before level L starts) and is cleared by level
// L's decide.
struct MsCtl {
  int32_t levels;  // levels run (for the caller; the kernel keeps its own count)
  int32_t pad;
  unsigned long long hcnt[2];
  alignas(128) unsigned long long acc[3][16];  // [0] new pairs, [1] frontier edges, [2] OR of new bits
};

constexpr size_t kMsCtlBytes = 1024;  // MsCtl, rounded up
constexpr int kMsMaxBlocks = 8192;
static_assert(sizeof(MsCtl) <= kMsCtlBytes, "control block too large");

template <class RowT>
struct MsArgs {
  const RowT *rp;
  const int32_t *col;
  int64_t n, nnz;
  uint64_t *seen, *front, *next;
  uint8_t *dist8;
  MsCtl *ctl;
  int32_t k;
  int32_t bu_percent;
  int32_t heavy;  // rows longer than this are handled by the whole wavefront
  int32_t aligned4;  // dist8 is 4-byte aligned
  uint64_t *hq;      // chunk queue of the rows longer than kMsChunk: chunk << 32 | v
  int64_t hq_cap;
  uint64_t *planes;  // [8][n] distance bit planes, or null: rows written per level
  int32_t src[64];   // the k sources (passed by value: no copy to the device first)
};

constexpr int kMsPlaneMinK = 16;

// Distance rows from the bit planes: lane = vertex v, one byte store per
// search, so a wavefront writes whole 64-byte row segments.  dmax is the
// largest distance written; plane b was written iff 2^b <= dmax, and NP
// planes cover dmax (NP = 8 also covers the saturated 255).
template <int NP, class RowT>
__device__ void ms_write_rows(const MsArgs<RowT> &A, int64_t v, int dmax) {
  const uint64_t s = A.seen[v];
  uint32_t lo[NP], hi[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const uint64_t p = (1 << b) <= dmax ? A.planes[(int64_t)b * A.n + v] : 0ull;
    lo[b] = (uint32_t)p;
    hi[b] = (uint32_t)(p >> 32);
  }
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    if (i >= A.k) break;
    const uint32_t *q = i < 32 ? lo : hi;
    const int sh = i & 31;
    uint32_t d = 0;
#pragma unroll
    for (int b = 0; b < NP; ++b) d |= ((q[b] >> sh) & 1u) << b;
    const uint8_t byte = ((s >> i) & 1ull) ? (uint8_t)d : (uint8_t)255;
    __builtin_nontemporal_store(byte, A.dist8 + (int64_t)i * A.n + v);
  }
}

// Top-down rows longer than kMsChunk edges are not walked by the wavefront
// that owns their vertex (a hub's row would take one dependent step per 64
// edges): a vertex with such a row queues its kMsChunk-edge chunks when it
// enters the frontier (at the start, or in the finalize pass of the level
// that finds it), and in a top-down level every wavefront takes chunks from
// the queue once its own words are done.  In the finalize pass a workgroup
// collects its long rows in LDS and reserves their queue entries with one
// atomic, so the queue counter sees one request per workgroup rather than
// one per hub.
constexpr int64_t kMsChunk = 1024;
constexpr int kMsHubList = 256;  // long rows a workgroup collects per level (more go straight to the queue)

template <class RowT>
__device__ void ms_queue_chunks(const MsArgs<RowT> &A, int64_t v, int64_t deg, unsigned long long *hcnt) {
  const uint64_t nch = (uint64_t)((deg + kMsChunk - 1) / kMsChunk);
  const unsigned long long base = atomicAdd(hcnt, (unsigned long long)nch);
  for (uint64_t k = 0; k < nch; ++k)
    if ((int64_t)(base + k) < A.hq_cap) A.hq[base + k] = (k << 32) | (uint32_t)v;
}

// Top-down expansion of the wavefront's 64 vertices starting at v0.
template <class RowT>
__device__ void ms_td(const MsArgs<RowT> &A, int64_t v0) {
  const int lane = lane_id();
  const int64_t v = v0 + lane;
  const uint64_t f = v < A.n ? A.front[v] : 0ull;
  int64_t beg = 0, end = 0;
  if (f) {
    beg = (int64_t)A.rp[v];
    end = (int64_t)A.rp[v + 1];
  }
  if (end - beg > kMsChunk) beg = end = 0;  // a long row: its chunks are queued
  const bool heavy = (end - beg) > A.heavy;
  if (f && !heavy) {
    for (int64_t j = beg; j < end; ++j) {
      const int32_t x = A.col[j];
      const uint64_t nb = f & ~A.seen[x];
      if (nb) atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), (unsigned long long)nb);
    }
  }
  uint64_t hm = __ballot(heavy);
  while (hm) {
    const int l = __ffsll((unsigned long long)hm) - 1;
    hm &= hm - 1;
    const int64_t b0 = __shfl(beg, l), e0 = __shfl(end, l);
    const uint64_t fl = __shfl(f, l);
    for (int64_t j = b0 + lane; j < e0; j += kWave) {
      const int32_t x = A.col[j];
      const uint64_t nb = fl & ~A.seen[x];
      if (nb) atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), (unsigned long long)nb);
    }
  }
}

// Bottom-up gathering for the wavefront's 64 vertices starting at v0.
template <class RowT>
__device__ void ms_bu(const MsArgs<RowT> &A, int64_t v0, uint64_t alive) {
  const int lane = lane_id();
  const int64_t v = v0 + lane;
  const uint64_t target = v < A.n ? (~A.seen[v] & alive) : 0ull;
  int64_t beg = 0, end = 0;
  if (target) {
    beg = (int64_t)A.rp[v];
    end = (int64_t)A.rp[v + 1];
  }
  const bool heavy = (end - beg) > A.heavy;
  uint64_t acc = 0;
  if (target && !heavy) {
    for (int64_t j = beg; j < end; ++j) {
      acc |= A.front[A.col[j]];
      if ((acc & target) == target) break;
    }
  }
  uint64_t hm = __ballot(heavy);
  while (hm) {
    const int l = __ffsll((unsigned long long)hm) - 1;
    hm &= hm - 1;
    const int64_t b0 = __shfl(beg, l), e0 = __shfl(end, l);
    const uint64_t tl = __shfl(target, l);
    uint64_t al = 0;
    for (int64_t b = b0; b < e0; b += kWave) {
      const int64_t j = b + lane;
      const uint64_t fr = j < e0 ? A.front[A.col[j]] : 0ull;
      al |= wave_or(fr);
      if ((al & tl) == tl) break;
    }
    if (lane == l) acc = al;
  }
  if (v < A.n) A.next[v] = acc & target;
}

template <class RowT>
__global__ void __launch_bounds__(1024) k_msbfs(MsArgs<RowT> A) {
  cg::grid_group grid = cg::this_grid();
  const int lane = lane_id();
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t wave = tid >> 6;
  const int64_t nwaves = nthreads >> 6;
  const int64_t nwords = (A.n + kWave - 1) / kWave;
  MsCtl *c = A.ctl;
  __shared__ unsigned long long part[3][16];
  __shared__ uint32_t hub_v[kMsHubList], hub_off[kMsHubList];
  __shared__ uint32_t hub_n, hub_chunks;
  __shared__ unsigned long long hub_base;
  if (threadIdx.x == 0) hub_n = hub_chunks = 0;

  // Initialisation: empty sets, every distance 255 (unreached).
  for (int64_t v = tid; v < A.n; v += nthreads) {
    A.seen[v] = 0;
    A.front[v] = 0;
    A.next[v] = 0;
  }
  const int64_t bytes = (int64_t)A.k * A.n;
  const int64_t head = A.aligned4 ? bytes / 4 : 0;  // 4-byte stores when the rows allow it
  uint32_t *d32 = reinterpret_cast<uint32_t *>(A.dist8);
  // (streaming stores: the rows are written once more, byte by byte, and
  // never read here)
  if (!A.planes) {
    for (int64_t i = tid; i < head; i += nthreads) __builtin_nontemporal_store(0xFFFFFFFFu, d32 + i);
    for (int64_t i = head * 4 + tid; i < bytes; i += nthreads) __builtin_nontemporal_store((uint8_t)255, A.dist8 + i);
  }
  if (tid == 0) {
    c->levels = 0;
    c->hcnt[0] = c->hcnt[1] = 0;
    for (int i = 0; i < 3; ++i) c->acc[i][0] = c->acc[i][1] = c->acc[i][2] = 0;
  }
  grid.sync();
  if (tid < A.k) {
    const int32_t s = A.src[tid];
    const unsigned long long bit = 1ull << tid;
    atomicOr(reinterpret_cast<unsigned long long *>(A.seen + s), bit);
    const uint64_t was = atomicOr(reinterpret_cast<unsigned long long *>(A.front + s), bit);
    const int64_t deg = (int64_t)A.rp[s + 1] - (int64_t)A.rp[s];
    if (was == 0 && deg > kMsChunk) ms_queue_chunks(A, s, deg, &c->hcnt[0]);
    if (!A.planes) A.dist8[(int64_t)tid * A.n + s] = 0;
  }
  grid.sync();

  int32_t dir = 0;  // 0 top-down, 1 bottom-up
  uint64_t alive = A.k == 64 ? ~0ull : ((1ull << A.k) - 1);  // searches whose frontier is not empty
  int dmax = (int)min(A.n + 1, (int64_t)255);                 // largest distance written
  for (int64_t level = 0; level <= A.n; ++level) {
    unsigned long long *hcnt = &c->hcnt[level & 1];
    for (int64_t w = wave; w < nwords; w += nwaves) {
      if (dir == 0)
        ms_td(A, w * kWave);
      else
        ms_bu(A, w * kWave, alive);
    }
    if (dir == 0) {  // the long rows' chunks, one per wavefront
      const int64_t nh = min((int64_t)__atomic_load_n(hcnt, __ATOMIC_RELAXED), A.hq_cap);
      for (int64_t i = wave; i < nh; i += nwaves) {
        const uint64_t e = A.hq[i];
        const int32_t v = (int32_t)(uint32_t)e;
        const uint64_t f = A.front[v];
        const int64_t b0 = (int64_t)A.rp[v] + (int64_t)(e >> 32) * kMsChunk;
        const int64_t e0 = min((int64_t)A.rp[v + 1], b0 + kMsChunk);
        for (int64_t j = b0 + lane; j < e0; j += kWave) {
          const int32_t x = A.col[j];
          const uint64_t nb = f & ~A.seen[x];
          if (nb) atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), (unsigned long long)nb);
        }
      }
    }
    grid.sync();
    // Finalize: next -> new frontier, seen, distance rows.
    const uint8_t dval = (uint8_t)(level + 1 < 255 ? level + 1 : 255);
    // planes: the first level whose distance sets bit b writes plane b in
    // full (so no plane is cleared beforehand); later ones OR into it
    unsigned long long pairs = 0, fedges = 0, bits = 0;
    for (int64_t w = wave; w < nwords; w += nwaves) {
      const int64_t v = w * kWave + lane;
      uint64_t nb = 0;
      if (v < A.n) {
        const uint64_t s = A.seen[v];
        nb = A.next[v] & ~s;
        A.next[v] = 0;
        A.front[v] = nb;
        if (nb) {
          A.seen[v] = s | nb;
          pairs += (unsigned long long)__popcll(nb);
          const int64_t deg = (int64_t)A.rp[v + 1] - (int64_t)A.rp[v];
          fedges += (unsigned long long)deg;
          bits |= nb;
          if (deg > kMsChunk) {  // a long row enters the frontier: collect it
            const uint32_t slot = atomicAdd(&hub_n, 1u);
            if (slot < (uint32_t)kMsHubList) {
              hub_v[slot] = (uint32_t)v;
              hub_off[slot] = atomicAdd(&hub_chunks, (uint32_t)((deg + kMsChunk - 1) / kMsChunk));
            } else {
              ms_queue_chunks(A, v, deg, &c->hcnt[(level + 1) & 1]);
            }
          }
        }
        if (A.planes) {
          for (int b = 0; b < 8; ++b) {
            if (!((dval >> b) & 1)) continue;
            uint64_t *pb = A.planes + (int64_t)b * A.n + v;
            if (dval == (1u << b))
              *pb = nb;
            else if (nb)
              *pb |= nb;
          }
        }
      }
      if (A.planes) continue;
      uint64_t any = wave_or(nb);
      while (any) {  // one coalesced byte row segment per search that advanced
        const int i = __ffsll((unsigned long long)any) - 1;
        any &= any - 1;
        if ((nb >> i) & 1ull) __builtin_nontemporal_store(dval, A.dist8 + (int64_t)i * A.n + v);
      }
    }
    __syncthreads();
    if (hub_n) {  // reserve the collected rows' chunks with one atomic, then write them
      if (threadIdx.x == 0) hub_base = atomicAdd(&c->hcnt[(level + 1) & 1], (unsigned long long)hub_chunks);
      __syncthreads();
      const uint32_t nl = min(hub_n, (uint32_t)kMsHubList);
      for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) {
        const int64_t v = hub_v[i];
        const int64_t deg = (int64_t)A.rp[v + 1] - (int64_t)A.rp[v];
        const uint64_t nch = (uint64_t)((deg + kMsChunk - 1) / kMsChunk);
        const unsigned long long at = hub_base + hub_off[i];
        for (uint64_t k = 0; k < nch; ++k)
          if ((int64_t)(at + k) < A.hq_cap) A.hq[at + k] = (k << 32) | (uint32_t)v;
      }
      __syncthreads();
      if (threadIdx.x == 0) hub_n = hub_chunks = 0;
    }
    pairs = wave_sum(pairs);
    fedges = wave_sum(fedges);
    bits = wave_or(bits);
    if (lane == 0) {
      part[0][threadIdx.x >> 6] = pairs;
      part[1][threadIdx.x >> 6] = fedges;
      part[2][threadIdx.x >> 6] = bits;
    }
    __syncthreads();
    unsigned long long *acc = c->acc[level % 3];
    if (threadIdx.x == 0) {  // this workgroup's totals into the level's accumulators
      unsigned long long p = 0, fe = 0, b = 0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        p += part[0][i];
        fe += part[1][i];
        b |= part[2][i];
      }
      if (p) {
        atomicAdd(&acc[0], p);
        atomicAdd(&acc[1], fe);
        atomicOr(&acc[2], b);
      }
    }
    grid.sync();
    const unsigned long long tp = __atomic_load_n(&acc[0], __ATOMIC_RELAXED);
    const unsigned long long tf = __atomic_load_n(&acc[1], __ATOMIC_RELAXED);
    const unsigned long long tb = __atomic_load_n(&acc[2], __ATOMIC_RELAXED);
    if (tid == 0) {
      unsigned long long *old = c->acc[(level + 2) % 3];
      old[0] = old[1] = old[2] = 0;
      *hcnt = 0;
      c->levels = (int32_t)(level + 1);
    }
    if (tp == 0) {
      dmax = (int)min(level + 1, (int64_t)255);
      break;
    }
    alive = tb;
    dir = (tf * 100ull > (unsigned long long)A.bu_percent * (unsigned long long)A.nnz) ? 1 : 0;
  }
  if (A.planes) {
    // the last level's distance bounds every distance; planes up to its top
    // bit were written
    for (int64_t v = tid; v < A.n; v += nthreads) {
      if (dmax < 16)
        ms_write_rows<4>(A, v, dmax);
      else
        ms_write_rows<8>(A, v, dmax);
    }
  }
}

// Where one batched search keeps its scratch.
struct MsView {
  uint64_t *seen, *front, *next, *hq, *planes;
  MsCtl *ctl;
  int64_t hq_cap;
};

// Every queued row has more than kMsChunk edges and enters a level's
// frontier once, so a level has fewer than 2 nnz / kMsChunk chunks.
int64_t ms_hq_cap(const bfs_graph *g) { return 2 * (g->nnz / kMsChunk) + 64; }

int ensure_ms_scratch(bfs_graph *g) {
  if (g->ms.seen) return BFS_OK;
  const size_t words = (size_t)g->n;
  const int64_t hq_cap = ms_hq_cap(g);
  void *p[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t sizes[6] = {words * 8, words * 8, words * 8, kMsCtlBytes,
                           (size_t)hq_cap * 8, 8 * words * 8};
  for (int i = 0; i < 6; ++i) {
    if (hipMalloc(&p[i], sizes[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(p[j]);
      return fail(BFS_ERR_OUT_OF_MEMORY, "cannot allocate batched-search scratch");
    }
  }
  g->ms.seen = static_cast<uint64_t *>(p[0]);
  g->ms.front = static_cast<uint64_t *>(p[1]);
  g->ms.next = static_cast<uint64_t *>(p[2]);
  g->ms.counters = static_cast<unsigned long long *>(p[3]);
  g->ms.hq = static_cast<uint64_t *>(p[4]);
  g->ms.hq_cap = hq_cap;
  g->ms.planes = static_cast<uint64_t *>(p[5]);
  g->ms.bytes = sizes[0] + sizes[1] + sizes[2] + sizes[3] + sizes[4] + sizes[5];
  return BFS_OK;
}

template <class RowT>
int batch_impl(bfs_graph *g, const MsView &V, const int32_t *sources, int32_t k, uint8_t *dist8, hipStream_t st) {
  MsArgs<RowT> A;
  A.rp = static_cast<const RowT *>(g->rp);
  A.col = g->col;
  A.n = g->n;
  A.nnz = g->nnz;
  A.seen = V.seen;
  A.front = V.front;
  A.next = V.next;
  A.dist8 = dist8;
  A.hq = V.hq;
  A.hq_cap = V.hq_cap;
  A.planes = k >= kMsPlaneMinK ? V.planes : nullptr;
  A.ctl = V.ctl;
  A.k = k;
  A.bu_percent = g->params.msbfs_bu_percent;
  A.heavy = kWave;
  A.aligned4 = (reinterpret_cast<uintptr_t>(dist8) & 3) == 0;
  for (int i = 0; i < 64; ++i) A.src[i] = i < k ? sources[i] : 0;
  const int bs = g->params.msbfs_block_size;
  int per_cu = 0, cus = 0;
  BFS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_msbfs<RowT>, bs, 0));
  BFS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  if (per_cu < 1) return fail(BFS_ERR_DEVICE, "batched kernel cannot be resident");
  const int blocks = std::min(per_cu * cus, kMsMaxBlocks);
  void *args[] = {&A};
  BFS_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_msbfs<RowT>), dim3(blocks),
                                     dim3(bs), args, 0, st));
  BFS_HIP(hipStreamSynchronize(st));
  return BFS_OK;
}

// Scratch of the allocation-free batched search: one file-scope device
// array per GPU, kept by the process until it ends.  Host code never uses
// the array's name as an address (on the host it names a stand-in, not
// device memory): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and is kept per device.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu[kMaxDevices];  // one search at a time per device uses its array
void *g_static_ptr[kMaxDevices];      // its device address, once taken (under the lock)

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the static array a batch of k searches on g uses (the layout of
// static_view).
size_t static_scratch_bytes(const bfs_graph *g, int32_t k) {
  const size_t sets = round256((size_t)g->n * 8);
  size_t b = 3 * sets + round256(kMsCtlBytes) + round256((size_t)ms_hq_cap(g) * 8);
  if (k >= kMsPlaneMinK) b += 8 * sets;
  return b;
}

MsView static_view(const bfs_graph *g, uint8_t *base, int32_t k) {
  const size_t sets = round256((size_t)g->n * 8);
  MsView V;
  size_t off = 0;
  V.seen = reinterpret_cast<uint64_t *>(base + off), off += sets;
  V.front = reinterpret_cast<uint64_t *>(base + off), off += sets;
  V.next = reinterpret_cast<uint64_t *>(base + off), off += sets;
  V.ctl = reinterpret_cast<MsCtl *>(base + off), off += round256(kMsCtlBytes);
  V.hq = reinterpret_cast<uint64_t *>(base + off), off += round256((size_t)ms_hq_cap(g) * 8);
  V.hq_cap = ms_hq_cap(g);
  V.planes = k >= kMsPlaneMinK ? reinterpret_cast<uint64_t *>(base + off) : nullptr;
  return V;
}

}  // namespace

int run_batch(bfs_graph *g, const int32_t *sources, int32_t k, uint8_t *dist8, hipStream_t stream) {
  hipStream_t st = stream ? stream : g->stream;
  int rc = ensure_ms_scratch(g);
  if (rc) return rc;
  MsView V;
  V.seen = g->ms.seen;
  V.front = g->ms.front;
  V.next = g->ms.next;
  V.hq = g->ms.hq;
  V.hq_cap = g->ms.hq_cap;
  V.planes = g->ms.planes;
  V.ctl = reinterpret_cast<MsCtl *>(g->ms.counters);
  return g->rp64 ? batch_impl<int64_t>(g, V, sources, k, dist8, st)
                 : batch_impl<int32_t>(g, V, sources, k, dist8, st);
}

int run_batch_static(bfs_graph *g, const int32_t *sources, int32_t k, uint8_t *dist8) {
  const size_t need = static_scratch_bytes(g, k);
  if (need > kStaticScratchBytes)
    return fail(BFS_ERR_INVALID_ARG,
                "the graph needs %zu bytes of batch scratch for k = %d; the allocation-free entry point "
                "holds %zu (use bfs_run_batch)", need, k, kStaticScratchBytes);
  if (g->device < 0 || g->device >= kMaxDevices)
    return fail(BFS_ERR_INVALID_ARG, "device %d beyond the %d the library tracks", g->device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_static_mu[g->device]);
  if (!g_static_ptr[g->device]) {  // first call on this device (which is current)
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BFS_ERR_DEVICE, "hipGetSymbolAddress of the batch scratch failed: %s", hipGetErrorString(e));
    g_static_ptr[g->device] = p;
  }
  const MsView V = static_view(g, static_cast<uint8_t *>(g_static_ptr[g->device]), k);
  return g->rp64 ? batch_impl<int64_t>(g, V, sources, k, dist8, g->stream)
                 : batch_impl<int32_t>(g, V, sources, k, dist8, g->stream);
}

}  // namespace bfsmi
