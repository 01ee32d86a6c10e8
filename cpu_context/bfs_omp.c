/*
 * OpenMP versions of the paper's CPU kernels (Section 2), as a multicore
 * context figure beside the GPU library and the serial oracle.  Not the
 * oracle (that is oracle/bfs_oracle.c, serial and plain) and not part of
 * the GPU library; written from the paper's descriptions:
 *
 *   omp_bfs(..., kind = 0)  BFS-Conventional: level-synchronous top-down
 *                           over a frontier array; a neighbour is claimed by
 *                           a compare-and-swap of its distance from -1; each
 *                           thread collects its discoveries in a private
 *                           buffer, merged into the next frontier after the
 *                           level.
 *   omp_bfs(..., kind = 1)  BFS-Hybrid (dagger): the same top-down step, and
 *                           a bottom-up step over the unvisited vertices that
 *                           stops at the first neighbour in the frontier;
 *                           the direction follows the alpha/beta rule
 *                           (top-down -> bottom-up when m_f * alpha > m_u,
 *                           back when n_f * beta < N and the frontier
 *                           shrinks), with the frontier converted between
 *                           the array and a bitmap at each switch.
 *   omp_bfs(..., kind = 2)  BFS-VisitedBitmap: BFS-Hybrid whose visited test
 *                           is a bitmap (one bit per vertex, claimed with an
 *                           atomic OR) instead of the distance array.
 *
 * Distances are written with plain stores by the claiming thread (every
 * writer of a vertex in a level writes the same value).  Parents follow the
 * Graph500 convention (parent[s] = s, -1 unreached).  Returns the number of
 * levels run; *secs gets the wall time from initialisation to the last
 * level.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void) {
  struct timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

typedef struct {
  int32_t *v;
  int64_t n, cap;
} Buf;

static void push(Buf *b, int32_t x) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 4096;
    b->v = (int32_t *)realloc(b->v, (size_t)b->cap * sizeof(int32_t));
  }
  b->v[b->n++] = x;
}

/* Claims v for this level: true for exactly one caller. */
static inline int claim(int kind, int32_t *dist, uint64_t *vis, int32_t v, int32_t d) {
  if (kind == 2) {
    const uint64_t bit = 1ull << (v & 63);
    if (__atomic_load_n(&vis[v >> 6], __ATOMIC_RELAXED) & bit) return 0;
    return !(__atomic_fetch_or(&vis[v >> 6], bit, __ATOMIC_RELAXED) & bit);
  }
  if (__atomic_load_n(&dist[v], __ATOMIC_RELAXED) != -1) return 0;
  return __sync_bool_compare_and_swap(&dist[v], -1, d);
}

int64_t omp_bfs(int64_t n, const int64_t *rp, const int32_t *col, int32_t s, int32_t kind, int32_t alpha,
                int32_t beta, int32_t threads, int32_t *dist, int32_t *parent, double *secs) {
  if (threads > 0) omp_set_num_threads(threads);
  const int64_t words = (n + 63) / 64;
  int32_t *front = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t *next = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  uint64_t *fbm = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* frontier bitmap */
  uint64_t *nbm = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* next frontier bitmap */
  uint64_t *vis = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* kind 2 only */
  const double t0 = now_s();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    dist[i] = -1;
    if (parent) parent[i] = -1;
  }
  dist[s] = 0;
  if (parent) parent[s] = s;
  if (kind == 2) vis[s >> 6] |= 1ull << (s & 63);
  int64_t nf = 1, mf = rp[s + 1] - rp[s];
  int64_t mu = rp[n] - mf;
  front[0] = s;
  int top_down = 1;      /* the current frontier is in `front` (else in fbm) */
  int64_t levels = 0;
  for (int32_t level = 0; nf > 0; ++level, ++levels) {
    int64_t found = 0, fdeg = 0;
    if (top_down) {
      int64_t nn = 0;
#pragma omp parallel reduction(+ : found, fdeg)
      {
        Buf b = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < nf; ++i) {
          const int32_t u = front[i];
          for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t v = col[e];
            if (claim(kind, dist, vis, v, level + 1)) {
              dist[v] = level + 1;
              if (parent) parent[v] = u;
              push(&b, v);
              fdeg += rp[v + 1] - rp[v];
            }
          }
        }
        found = b.n;
        const int64_t at = __atomic_fetch_add(&nn, b.n, __ATOMIC_RELAXED);
        if (b.n) memcpy(next + at, b.v, (size_t)b.n * sizeof(int32_t));
        free(b.v);
      }
      int32_t *t = front;
      front = next;
      next = t;
    } else {
      /* bottom-up: every unvisited vertex looks for a neighbour in the
         frontier; a thread owns whole 64-vertex words of the next bitmap */
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : found, fdeg)
      for (int64_t w = 0; w < words; ++w) {
        uint64_t out = 0;
        for (int64_t v = w * 64; v < (w + 1) * 64 && v < n; ++v) {
          const int unvisited = kind == 2 ? !((vis[w] >> (v & 63)) & 1ull) : dist[v] == -1;
          if (!unvisited) continue;
          for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t x = col[e];
            if ((fbm[x >> 6] >> (x & 63)) & 1ull) {
              dist[v] = level + 1;
              if (parent) parent[v] = x;
              out |= 1ull << (v & 63);
              ++found;
              fdeg += rp[v + 1] - rp[v];
              break;
            }
          }
        }
        nbm[w] = out;
        if (kind == 2) vis[w] |= out;
      }
      uint64_t *t = fbm;
      fbm = nbm;
      nbm = t;
    }
    /* direction for the next level (alpha/beta rule; kind 0 stays top-down) */
    mu -= fdeg;
    int next_td = 1;
    if (kind != 0) {
      if (top_down) next_td = !(fdeg * (int64_t)alpha > mu);
      else next_td = found * (int64_t)beta < n && found < nf;
    }
    if (found > 0 && next_td != top_down) {
      if (next_td) { /* bitmap -> array */
        int64_t nn = 0;
#pragma omp parallel
        {
          Buf b = {0, 0, 0};
#pragma omp for schedule(static)
          for (int64_t w = 0; w < words; ++w)
            for (uint64_t m = fbm[w]; m; m &= m - 1) push(&b, (int32_t)(w * 64 + __builtin_ctzll(m)));
          const int64_t at = __atomic_fetch_add(&nn, b.n, __ATOMIC_RELAXED);
          if (b.n) memcpy(front + at, b.v, (size_t)b.n * sizeof(int32_t));
          free(b.v);
        }
      } else { /* array -> bitmap */
#pragma omp parallel for schedule(static)
        for (int64_t w = 0; w < words; ++w) fbm[w] = 0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < found; ++i)
          __atomic_fetch_or(&fbm[front[i] >> 6], 1ull << (front[i] & 63), __ATOMIC_RELAXED);
      }
      top_down = next_td;
    }
    nf = found;
    mf = fdeg;
    (void)mf;
  }
  *secs = now_s() - t0;
  free(front);
  free(next);
  free(fbm);
  free(nbm);
  free(vis);
  return levels;
}
