// Optional preprocessing at graph creation: reorders every row so that
// higher-degree neighbours come first (ties keep ascending ids).
//
// A bottom-up level (Section 2, BFS-Hybrid) stops scanning a vertex's row at
// the first neighbour found in the frontier.  In power-law graphs the large
// frontiers are made of high-degree vertices, so listing them first makes
// the first hit come earlier; the distances do not change (only the order in
// which neighbours are examined, and so which valid parent is recorded).
//
// The sort key of a neighbour x is the 64-bit value (~deg(x) << 32) | x:
// ascending keys give descending degree, then ascending id, and the key
// carries the id itself, so a row is sorted by sorting its keys alone.
// Rows are sorted in three classes by length:
//   2..64       a wavefront per row, one key per lane, a bitonic network of
//               lane exchanges (registers only);
//   65..4096    a workgroup per row, a bitonic network in LDS;
//   > 4096      a workgroup per row: 4096-key runs sorted in LDS, then
//               merged pairwise in global memory, each thread producing an
//               equal share of every merged pair (its start found by a
//               binary search along the merge path).
// Runs once, when the graph is created; the head records are rebuilt after.

#include <algorithm>

#include "common.h"
#include "device_util.h"

namespace bfsmi {
namespace {

constexpr int kMidMax = 4096;   // longest row sorted in one LDS tile
constexpr int kSortBlock = 256;

__device__ __forceinline__ uint64_t sort_key(const int4 *head, int32_t x) {
  return ((uint64_t)(~(uint32_t)head[x].x) << 32) | (uint32_t)x;
}

// Compare-exchange of a bitonic network over 64 lanes: stage (k, j).
__device__ __forceinline__ uint64_t lane_cmpx(uint64_t key, int lane, int k, int j) {
  const uint32_t lo = __shfl_xor((uint32_t)key, j);
  const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), j);
  const uint64_t other = ((uint64_t)hi << 32) | lo;
  const bool up = (lane & k) == 0;          // this 2k-block sorts ascending
  const bool low = (lane & j) == 0;         // this lane keeps the smaller of the pair (if ascending)
  const uint64_t mn = key < other ? key : other, mx = key < other ? other : key;
  return (up == low) ? mn : mx;
}

// Rows of 2..64 entries: one row per wavefront at a time.
template <class RowT>
__global__ void __launch_bounds__(kSortBlock) k_sort_short(const RowT *rp, int32_t *col, const int4 *head,
                                                            int64_t n) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int64_t b = (int64_t)rp[v], len = (int64_t)rp[v + 1] - b;
    if (len < 2 || len > kWave) continue;  // uniform over the wavefront
    uint64_t key = lane < len ? sort_key(head, col[b + lane]) : ~0ull;
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) key = lane_cmpx(key, lane, k, j);
    if (lane < len) col[b + lane] = (int32_t)(uint32_t)key;
  }
}

// Bitonic sort of `p` keys (a power of two, <= kMidMax) in LDS by the
// calling workgroup; every thread calls it.
__device__ void lds_bitonic(uint64_t *t, int p) {
  for (int k = 2; k <= p; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < p; i += blockDim.x) {
        const int q = i ^ j;
        if (q > i) {
          const uint64_t a = t[i], c = t[q];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            t[i] = c;
            t[q] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Loads `len` keys of the row segment starting at col + b into LDS (padded
// with the largest key up to the power of two p), sorts them.
__device__ int lds_sort_segment(uint64_t *t, const int32_t *col, const int4 *head, int64_t b, int len) {
  int p = 2;
  while (p < len) p <<= 1;
  for (int i = threadIdx.x; i < p; i += blockDim.x) t[i] = i < len ? sort_key(head, col[b + i]) : ~0ull;
  __syncthreads();
  lds_bitonic(t, p);
  return p;
}

// Rows of 65..kMidMax entries, listed in `rows`: a workgroup per row.
template <class RowT>
__global__ void __launch_bounds__(kSortBlock) k_sort_mid(const RowT *rp, int32_t *col, const int4 *head,
                                                          const int32_t *rows, int64_t nrows) {
  __shared__ uint64_t t[kMidMax];
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t v = rows[r];
    const int64_t b = (int64_t)rp[v];
    const int len = (int)((int64_t)rp[v + 1] - b);
    lds_sort_segment(t, col, head, b, len);
    for (int i = threadIdx.x; i < len; i += blockDim.x) col[b + i] = (int32_t)(uint32_t)t[i];
    __syncthreads();
  }
}

// First index i of a (length la) such that the merged output's first d
// entries take i from a and d - i from b (ties taken from a first).
__device__ __forceinline__ int64_t merge_path(const uint64_t *a, int64_t la, const uint64_t *b, int64_t lb,
                                              int64_t d) {
  int64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= b[d - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Rows longer than kMidMax, listed in `rows` with their offsets `toff` into
// the two key buffers t0 / t1 (one entry per row entry each): a workgroup
// per row sorts its kMidMax-key runs in LDS, merges them pairwise between
// the buffers, and writes the ids back.
template <class RowT>
__global__ void __launch_bounds__(kSortBlock) k_sort_long(const RowT *rp, int32_t *col, const int4 *head,
                                                           const int32_t *rows, const int64_t *toff,
                                                           int64_t nrows, uint64_t *t0, uint64_t *t1) {
  __shared__ uint64_t t[kMidMax];
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t v = rows[r];
    const int64_t b = (int64_t)rp[v];
    const int64_t len = (int64_t)rp[v + 1] - b;
    uint64_t *src = t0 + toff[r], *dst = t1 + toff[r];
    for (int64_t c = 0; c < len; c += kMidMax) {
      const int cl = (int)min((int64_t)kMidMax, len - c);
      lds_sort_segment(t, col, head, b + c, cl);
      for (int i = threadIdx.x; i < cl; i += blockDim.x) src[c + i] = t[i];
      __syncthreads();
    }
    for (int64_t w = kMidMax; w < len; w <<= 1) {  // runs of w keys -> runs of 2w
      for (int64_t a0 = 0; a0 < len; a0 += 2 * w) {
        const int64_t la = min(w, len - a0);
        const int64_t lb = min(w, len - a0 - la);
        const uint64_t *A = src + a0, *B = src + a0 + la;
        uint64_t *out = dst + a0;
        const int64_t tot = la + lb;
        const int64_t per = (tot + blockDim.x - 1) / blockDim.x;
        const int64_t d0 = min(tot, (int64_t)threadIdx.x * per), d1 = min(tot, d0 + per);
        int64_t i = merge_path(A, la, B, lb, d0), j = d0 - i;
        for (int64_t d = d0; d < d1; ++d) {
          if (j >= lb || (i < la && A[i] <= B[j]))
            out[d] = A[i++];
          else
            out[d] = B[j++];
        }
      }
      // the barrier makes this pass's global writes visible to the whole
      // workgroup before the next pass reads them
      __syncthreads();
      uint64_t *x = src;
      src = dst;
      dst = x;
    }
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) col[b + i] = (int32_t)(uint32_t)src[i];
    __syncthreads();
  }
}

template <class RowT>
int sort_rows(bfs_graph *g, const int64_t *host_rp) {
  const int64_t nnz = g->nnz, n = g->n;
  if (nnz == 0) return BFS_OK;
  if (nnz >= ((int64_t)1 << 31)) return fail(BFS_ERR_INVALID_ARG, "BFS_SORT_NEIGHBORS needs nnz < 2^31");
  // rows of the two workgroup classes, from the host copy of the offsets
  std::vector<int32_t> mid, lng;
  std::vector<int64_t> toff;
  int64_t tlen = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t len = host_rp[v + 1] - host_rp[v];
    if (len > kMidMax) {
      lng.push_back((int32_t)v);
      toff.push_back(tlen);
      tlen += len;
    } else if (len > kWave) {
      mid.push_back((int32_t)v);
    }
  }
  int32_t *d_mid = nullptr, *d_lng = nullptr;
  int64_t *d_toff = nullptr;
  uint64_t *t0 = nullptr, *t1 = nullptr;
  auto cleanup = [&]() {
    for (void *p : {(void *)d_mid, (void *)d_lng, (void *)d_toff, (void *)t0, (void *)t1})
      if (p) (void)hipFree(p);
  };
  hipError_t e = hipSuccess;
  if (!mid.empty()) e = hipMalloc((void **)&d_mid, sizeof(int32_t) * mid.size());
  if (e == hipSuccess && !lng.empty()) e = hipMalloc((void **)&d_lng, sizeof(int32_t) * lng.size());
  if (e == hipSuccess && !lng.empty()) e = hipMalloc((void **)&d_toff, sizeof(int64_t) * toff.size());
  if (e == hipSuccess && tlen > 0) e = hipMalloc((void **)&t0, sizeof(uint64_t) * tlen);
  if (e == hipSuccess && tlen > 0) e = hipMalloc((void **)&t1, sizeof(uint64_t) * tlen);
  if (e != hipSuccess) {
    cleanup();
    return fail(BFS_ERR_OUT_OF_MEMORY, "no device memory to reorder rows");
  }
  if (!mid.empty()) e = hipMemcpy(d_mid, mid.data(), sizeof(int32_t) * mid.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !lng.empty())
    e = hipMemcpy(d_lng, lng.data(), sizeof(int32_t) * lng.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !lng.empty())
    e = hipMemcpy(d_toff, toff.data(), sizeof(int64_t) * toff.size(), hipMemcpyHostToDevice);
  const RowT *rp = static_cast<const RowT *>(g->rp);
  if (e == hipSuccess) {
    const int blocks = (int)std::min<int64_t>((n + (kSortBlock / kWave) - 1) / (kSortBlock / kWave), 65536);
    hipLaunchKernelGGL(k_sort_short<RowT>, dim3(blocks), dim3(kSortBlock), 0, nullptr, rp, g->col, g->head, n);
    if (!mid.empty())
      hipLaunchKernelGGL(k_sort_mid<RowT>, dim3((unsigned)std::min<size_t>(mid.size(), 65536)), dim3(kSortBlock),
                         0, nullptr, rp, g->col, g->head, d_mid, (int64_t)mid.size());
    if (!lng.empty())
      hipLaunchKernelGGL(k_sort_long<RowT>, dim3((unsigned)std::min<size_t>(lng.size(), 65536)), dim3(kSortBlock),
                         0, nullptr, rp, g->col, g->head, d_lng, d_toff, (int64_t)lng.size(), t0, t1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  if (e != hipSuccess) return fail(BFS_ERR_DEVICE, "row reordering failed: %s", hipGetErrorString(e));
  return build_head(g);  // the first three neighbours changed
}

}  // namespace

int sort_neighbors_by_degree(bfs_graph *g, const int64_t *host_rp) {
  return g->rp64 ? sort_rows<int64_t>(g, host_rp) : sort_rows<int32_t>(g, host_rp);
}

}  // namespace bfsmi
