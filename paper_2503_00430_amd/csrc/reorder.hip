// Optional preprocessing at graph creation: reorders every row so that
// higher-degree neighbours come first (ties keep ascending ids).
//
// A bottom-up level (Section 2, BFS-Hybrid) stops scanning a vertex's row at
// the first neighbour found in the frontier.  In power-law graphs the large
// frontiers are made of high-degree vertices, so listing them first makes
// the first hit come earlier; the distances do not change (only the order in
// which neighbours are examined, and so which valid parent is recorded).
//
// Implementation: keys = degree of each neighbour, a stable descending
// segmented radix sort over rows (hipCUB), then the head records are
// rebuilt.  Runs once, when the graph is created.

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace bfsmi {
namespace {

__global__ void k_neighbor_degree(const int32_t *col, const int4 *head, uint32_t *key, int64_t nnz) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += stride)
    key[j] = (uint32_t)head[col[j]].x;
}

template <class RowT>
int sort_rows(bfs_graph *g) {
  const int64_t nnz = g->nnz;
  if (nnz == 0) return BFS_OK;
  if (nnz >= ((int64_t)1 << 31)) return fail(BFS_ERR_INVALID_ARG, "BFS_SORT_NEIGHBORS needs nnz < 2^31");
  uint32_t *kin = nullptr, *kout = nullptr;
  int32_t *vout = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  auto cleanup = [&]() {
    if (kin) (void)hipFree(kin);
    if (kout) (void)hipFree(kout);
    if (vout) (void)hipFree(vout);
    if (tmp) (void)hipFree(tmp);
  };
  if (hipMalloc((void **)&kin, sizeof(uint32_t) * nnz) != hipSuccess ||
      hipMalloc((void **)&kout, sizeof(uint32_t) * nnz) != hipSuccess ||
      hipMalloc((void **)&vout, sizeof(int32_t) * nnz) != hipSuccess) {
    cleanup();
    return fail(BFS_ERR_OUT_OF_MEMORY, "no device memory to reorder rows");
  }
  const int bs = 256;
  const int blocks = (int)std::min<int64_t>((nnz + bs - 1) / bs, 65536);
  hipLaunchKernelGGL(k_neighbor_degree, dim3(blocks), dim3(bs), 0, nullptr, g->col, g->head, kin, nnz);
  const RowT *off = static_cast<const RowT *>(g->rp);
  hipError_t e = hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, tmp_bytes, kin, kout, g->col, vout, (int)nnz, (int)g->n, off, off + 1, 0, 32, nullptr);
  if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 8));
  if (e == hipSuccess)
    e = hipcub::DeviceSegmentedRadixSort::SortPairsDescending(tmp, tmp_bytes, kin, kout, g->col, vout,
                                                              (int)nnz, (int)g->n, off, off + 1, 0, 32,
                                                              nullptr);
  if (e == hipSuccess) e = hipMemcpy(g->col, vout, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  cleanup();
  if (e != hipSuccess) return fail(BFS_ERR_DEVICE, "row reordering failed: %s", hipGetErrorString(e));
  return build_head(g);  // the first three neighbours changed
}

}  // namespace

int sort_neighbors_by_degree(bfs_graph *g) {
  return g->rp64 ? sort_rows<int64_t>(g) : sort_rows<int32_t>(g);
}

}  // namespace bfsmi
