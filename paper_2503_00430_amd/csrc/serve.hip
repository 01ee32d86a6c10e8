// Serving runtime (placeholder until the continuous-batching server lands).
#include "common.h"

using namespace bfsmi;

extern "C" {
int bfs_serve_create(size_t, int32_t, bfs_server_t *out) {
  if (out) *out = nullptr;
  return fail(BFS_ERR_DEVICE, "serving is not available in this build");
}
int bfs_serve_destroy(bfs_server_t) { return fail(BFS_ERR_INVALID_ARG, "null server"); }
int bfs_serve_submit(bfs_server_t, bfs_graph_t, int32_t, int32_t *, int32_t *, uint64_t *) {
  return fail(BFS_ERR_INVALID_ARG, "null server");
}
int bfs_serve_poll(bfs_server_t, uint64_t, int32_t *, bfs_req_stats *) {
  return fail(BFS_ERR_INVALID_ARG, "null server");
}
}
