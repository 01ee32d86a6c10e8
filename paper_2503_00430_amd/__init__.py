"""Python binding of libbfs (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/bfs.h).  PyTorch supplies device memory (output tensors) and
streams; all graph work runs in the library's HIP kernels.  The library
must be built (`python -m paper_2503_00430_amd.build`); importing fails
loudly when it is missing.
"""
from ._lib import (  # noqa: F401
    BFS_OK, BFS_ERR_INVALID_ARG, BFS_ERR_OUT_OF_MEMORY, BFS_ERR_DEVICE, BFS_ERR_BUSY, BFS_ERR_NOT_READY,
    BFS_INPUT_DEVICE, BFS_VALIDATE, BFS_VALIDATE_SYMMETRY, BFS_ROWPTR32, BFS_SORT_NEIGHBORS,
    BFS_POLICY_AUTO, BFS_POLICY_ALPHA_BETA, BFS_POLICY_FRONTIER_5PCT, BFS_POLICY_TD_ONLY,
    BFS_LOOP_AUTO, BFS_LOOP_HOST, BFS_LOOP_GRAPH, BFS_LOOP_PERSISTENT, BFS_LOOP_QUEUED,
    BFS_TD_VISITED_BITMAP, BFS_TD_DIST_CAS, BFS_TD_DIST_PLAIN, BFS_TD_DIST_PLAIN_CULL,
    BFS_REQ_QUEUED, BFS_REQ_RUNNING, BFS_REQ_DONE, BFS_REQ_FAILED,
    BfsError, Graph, Server, library_path, load_library,
    bfs_create_graph, bfs_destroy_graph, bfs_graph_set_stream, bfs_graph_copy_csr, bfs_set_params, bfs_get_params,
    bfs_default_params, bfs_graph_info_get, bfs_run, bfs_get_run_stats, bfs_run_batch,
    bfs_run_batch_noalloc, BFS_NOALLOC_SCRATCH_BYTES,
    bfs_serve_create, bfs_serve_destroy, bfs_serve_submit, bfs_serve_poll, bfs_last_error,
)
