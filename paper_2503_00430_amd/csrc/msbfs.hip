// Batched multi-source BFS (placeholder until the persistent kernel lands).
#include "common.h"

namespace bfsmi {
int run_batch(bfs_graph *, const int32_t *, int32_t, uint8_t *, hipStream_t) {
  return fail(BFS_ERR_DEVICE, "bfs_run_batch is not available in this build");
}
}  // namespace bfsmi
