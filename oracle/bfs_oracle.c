/*
 * Serial breadth-first search over a CSR graph -- the CHECKER for the GPU
 * library.  Test infrastructure only: the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the library never does.
 *
 * What it computes (the paper's problem statement, Section 1, and the
 * output of every kernel variant in Section 2, Listings 1-3): for a source
 * s, dist[v] is the number of edges on a shortest s-v path, or -1 when v is
 * not reachable from s.  This is the textbook FIFO-queue BFS, written with
 * no blocking, no parallelism and no direction switching, so that it can be
 * checked against the definition by eye.
 *
 * parent[] follows the usual BFS-tree convention (the paper has no parents):
 * parent[s] = s, parent[v] = the vertex whose expansion first reached v,
 * -1 when unreached.  Parents are not unique in general; the GPU side is
 * checked against invariants, not against these values.
 *
 * Built with ORACLE_MUTANT=k it compiles a deliberately wrong variant, used
 * only by the tests that show the pins catch such mistakes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <time.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

static double now_seconds(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Single-source BFS.  row_ptr has n+1 entries, col has row_ptr[n] entries.
 * dist[n] is required, parent[n] may be NULL.  *seconds (if not NULL)
 * receives the wall time of initialisation plus traversal.
 * Returns the number of reached vertices, or -1 on bad arguments or
 * allocation failure.
 */
int64_t oracle_bfs(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t source,
                   int32_t *dist, int32_t *parent, double *seconds) {
  if (n < 1 || source < 0 || source >= n || !row_ptr || !col || !dist) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -1;
  double t0 = now_seconds();
  for (int64_t v = 0; v < n; ++v) dist[v] = -1;
  if (parent)
    for (int64_t v = 0; v < n; ++v) parent[v] = -1;
  int64_t head = 0, tail = 0;
#if ORACLE_MUTANT == 5
  dist[source] = 1; /* mutant: source not at distance zero */
#else
  dist[source] = 0;
#endif
  if (parent) parent[source] = source;
  queue[tail++] = source;
  while (head < tail) {
#if ORACLE_MUTANT == 1
    int32_t u = queue[--tail]; /* mutant: LIFO stack, i.e. depth-first order */
    if (tail < head) break;
#else
    int32_t u = queue[head++];
#endif
#if ORACLE_MUTANT == 4
    int64_t end = row_ptr[u + 1] - 1; /* mutant: last neighbour never examined */
#else
    int64_t end = row_ptr[u + 1];
#endif
    for (int64_t j = row_ptr[u]; j < end; ++j) {
      int32_t v = col[j];
      if (dist[v] < 0) {
#if ORACLE_MUTANT == 2
        dist[v] = dist[u]; /* mutant: dropped +1 */
#elif ORACLE_MUTANT == 6
        dist[v] = dist[u] + 1 + (dist[u] > 2); /* mutant: wrong beyond level 3 */
#else
        dist[v] = dist[u] + 1;
#endif
#if ORACLE_MUTANT == 3
        if (parent) parent[v] = v; /* mutant: wrong index stored as parent */
#else
        if (parent) parent[v] = u;
#endif
        queue[tail++] = v;
      }
    }
  }
  double t1 = now_seconds();
  if (seconds) *seconds = t1 - t0;
  free(queue);
#if ORACLE_MUTANT == 1
  {
    int64_t reached = 0;
    for (int64_t v = 0; v < n; ++v) reached += dist[v] >= 0;
    return reached;
  }
#else
  return tail;
#endif
}

/*
 * Work profile of one bottom-up level (Section 2, BFS-Hybrid bottom-up
 * step), derived from a finished distance array.  Level L expands the
 * frontier F = {v : dist[v] == L}.  The vertices still unvisited when level
 * L runs are U = {v : dist[v] == -1 or dist[v] > L}.  Each u in U examines
 * its neighbours in CSR order and stops at the first one in F; e_u is the
 * number of neighbours examined (1 + index of the first hit, or deg(u) when
 * none is in F).
 *
 * out[0] = |U| restricted to vertices of nonzero degree
 * out[1] = sum of e_u over U
 * out[2] = number of u in U that find a frontier neighbour (= |{dist == L+1}|)
 * out[3] = sum of deg(u) over U (edges a scan without early exit would read)
 */
void oracle_bottom_up_profile(int64_t n, const int64_t *row_ptr, const int32_t *col,
                              const int32_t *dist, int32_t level, int64_t *out) {
  int64_t unvisited = 0, examined = 0, found = 0, full = 0;
  for (int64_t u = 0; u < n; ++u) {
    if (!(dist[u] < 0 || dist[u] > level)) continue;
    int64_t beg = row_ptr[u], end = row_ptr[u + 1];
    if (end == beg) continue;
    ++unvisited;
    full += end - beg;
    int64_t e = end - beg;
    for (int64_t j = beg; j < end; ++j) {
      if (dist[col[j]] == level) {
        e = j - beg + 1;
        ++found;
        break;
      }
    }
    examined += e;
  }
  out[0] = unvisited;
  out[1] = examined;
  out[2] = found;
  out[3] = full;
}

/*
 * Check of a BFS tree (the parent convention above) against a distance
 * array that is already known to be exact.  For every vertex v it tests
 *   out[0]  P1: parent[source] == source;
 *   out[1]  P3: parent[v] == -1 exactly when dist[v] == -1;
 *   out[2]  P2: for reached v != source, parent[v] is a vertex id whose
 *               distance is dist[v] - 1;
 *   out[3]  P2: for reached v != source, parent[v] occurs in row v (the pair
 *               is an edge).
 * Each out[k] counts the vertices that violate it; out[4] is the first such
 * vertex (or -1).  One pass over the rows of the reached vertices.
 */
void oracle_check_tree(int64_t n, const int64_t *row_ptr, const int32_t *col, int32_t source,
                       const int32_t *dist, const int32_t *parent, int64_t *out) {
  int64_t bad[4] = {0, 0, 0, 0};
  int64_t first = -1;
  for (int64_t v = 0; v < n; ++v) {
    int viol = 0;
    const int32_t p = parent[v];
    if (v == source) {
      if (p != source) { ++bad[0]; viol = 1; }
    } else if (dist[v] < 0) {
      if (p != -1) { ++bad[1]; viol = 1; }
    } else if (p == -1) {
      ++bad[1]; viol = 1;
    } else if (p < -1 || p >= n || dist[p] != dist[v] - 1) {
      ++bad[2]; viol = 1;
    } else {
      int edge = 0;
      for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j)
        if (col[j] == p) { edge = 1; break; }
      if (!edge) { ++bad[3]; viol = 1; }
    }
    if (viol && first < 0) first = v;
  }
  for (int k = 0; k < 4; ++k) out[k] = bad[k];
  out[4] = first;
}
