/*
 * OpenMP versions of the paper's CPU kernels (Section 2), as a multicore
 * context figure beside the GPU library and the serial oracle.  Not the
 * oracle (that is oracle/bfs_oracle.c, serial and plain) and not part of
 * the GPU library; written from the paper's descriptions.
 *
 * A search is level-synchronous.  Two choices make the variants:
 *
 *   body (how a top-down step tells and claims an unvisited neighbour)
 *     BODY_CAS     compare-and-swap of the neighbour's distance from -1
 *                  (BFS-Conventional);
 *     BODY_PLAIN   a plain test of the distance and a plain store of the new
 *                  level (BFS-NonAtomic): racing threads may both pass the
 *                  test, so a vertex can enter the next frontier more than
 *                  once; every copy is expanded at the next level (all
 *                  writers store the same level, so the distances stay
 *                  exact);
 *     BODY_BITMAP  one bit per vertex, claimed with an atomic OR
 *                  (BFS-VisitedBitmap; a packed bit set by a plain
 *                  read-modify-write could be lost, see the library's
 *                  design notes).
 *   rule (direction of the next level, chosen after each level)
 *     RULE_TD_ONLY     top-down at every level;
 *     RULE_5PCT        bottom-up exactly when the new frontier holds at least
 *                      5 % of the vertices, 20 * n_f >= N (BFS-Hybrid);
 *     RULE_ALPHA_BETA  from top-down to bottom-up when m_f * alpha > m_u, back
 *                      when n_f * beta < N and the frontier shrank
 *                      (BFS-Hybrid dagger).
 * n_f is the frontier as the top-down step leaves it, duplicates included
 * for BODY_PLAIN (the merged thread-local frontiers the paper's test reads).
 *
 * Each thread collects its discoveries in a private buffer; the buffers are
 * merged into the next frontier array after the level.  The bottom-up step
 * gives each thread whole 64-vertex words of the next-frontier bitmap, and
 * every unvisited vertex stops at its first neighbour in the frontier.  The
 * frontier is converted between array and bitmap at each switch.
 *
 * Parents follow the Graph500 convention (parent[s] = s, -1 unreached).
 * Returns the number of levels run; *secs gets the wall time from
 * initialisation to the last level; *entries (if not NULL) the frontier
 * entries over all levels, duplicates included.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { BODY_CAS = 0, BODY_PLAIN = 1, BODY_BITMAP = 2 };
enum { RULE_TD_ONLY = 0, RULE_5PCT = 1, RULE_ALPHA_BETA = 2 };

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

/* Top-down claim of v for level d by the calling thread. */
static inline int claim(int body, int32_t *dist, uint64_t *vis, int32_t v, int32_t d) {
  if (body == BODY_BITMAP) {
    const uint64_t bit = 1ull << (v & 63);
    if (__atomic_load_n(&vis[v >> 6], __ATOMIC_RELAXED) & bit) return 0;
    return !(__atomic_fetch_or(&vis[v >> 6], bit, __ATOMIC_RELAXED) & bit);
  }
  if (body == BODY_PLAIN) {
    /* plain load and store (relaxed atomics compile to ordinary moves) */
    if (__atomic_load_n(&dist[v], __ATOMIC_RELAXED) != -1) return 0;
    __atomic_store_n(&dist[v], d, __ATOMIC_RELAXED);
    return 1;
  }
  if (__atomic_load_n(&dist[v], __ATOMIC_RELAXED) != -1) return 0;
  return __sync_bool_compare_and_swap(&dist[v], -1, d);
}

int64_t omp_bfs(int64_t n, const int64_t *rp, const int32_t *col, int32_t s, int32_t body, int32_t rule,
                int32_t alpha, int32_t beta, int32_t threads, int32_t *dist, int32_t *parent, double *secs,
                int64_t *entries) {
  if (threads > 0) omp_set_num_threads(threads);
  const int64_t words = (n + 63) / 64;
  int64_t fcap = n > 0 ? n : 1, ncap = fcap;  /* frontier arrays grow past n with duplicates */
  int32_t *front = (int32_t *)malloc((size_t)fcap * sizeof(int32_t));
  int32_t *next = (int32_t *)malloc((size_t)ncap * sizeof(int32_t));
  uint64_t *fbm = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* frontier bitmap */
  uint64_t *nbm = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* next frontier bitmap */
  uint64_t *vis = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));  /* BODY_BITMAP only */
  int64_t total_entries = 0;
  const double t0 = now_s();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    dist[i] = -1;
    if (parent) parent[i] = -1;
  }
  dist[s] = 0;
  if (parent) parent[s] = s;
  if (body == BODY_BITMAP) vis[s >> 6] |= 1ull << (s & 63);
  int64_t nf = 1;
  int64_t mu = rp[n] - (rp[s + 1] - rp[s]);
  front[0] = s;
  int top_down = 1; /* the current frontier is in `front` (else in fbm) */
  int64_t levels = 0;
  for (int32_t level = 0; nf > 0; ++level, ++levels) {
    total_entries += nf;
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
            if (claim(body, dist, vis, v, level + 1)) {
              /* (the bitmap claim leaves the distance to its winner) */
              if (body == BODY_BITMAP) __atomic_store_n(&dist[v], level + 1, __ATOMIC_RELAXED);
              if (parent) __atomic_store_n(&parent[v], u, __ATOMIC_RELAXED);
              push(&b, v);
              fdeg += rp[v + 1] - rp[v];
            }
          }
        }
        found = b.n;
        const int64_t at = __atomic_fetch_add(&nn, b.n, __ATOMIC_RELAXED);
#pragma omp barrier
#pragma omp single
        if (nn > ncap) {
          ncap = nn;
          next = (int32_t *)realloc(next, (size_t)ncap * sizeof(int32_t));
        }
        if (b.n) memcpy(next + at, b.v, (size_t)b.n * sizeof(int32_t));
        free(b.v);
      }
      int32_t *t = front;
      front = next;
      next = t;
      int64_t c = fcap;
      fcap = ncap;
      ncap = c;
    } else {
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : found, fdeg)
      for (int64_t w = 0; w < words; ++w) {
        uint64_t out = 0;
        for (int64_t v = w * 64; v < (w + 1) * 64 && v < n; ++v) {
          const int unvisited = body == BODY_BITMAP ? !((vis[w] >> (v & 63)) & 1ull) : dist[v] == -1;
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
        if (body == BODY_BITMAP) vis[w] |= out;
      }
      uint64_t *t = fbm;
      fbm = nbm;
      nbm = t;
    }
    mu -= fdeg;
    int next_td = 1;
    if (rule == RULE_5PCT) {
      next_td = !(20 * found >= n);
    } else if (rule == RULE_ALPHA_BETA) {
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
#pragma omp barrier
          if (b.n) memcpy(front + at, b.v, (size_t)b.n * sizeof(int32_t));
          free(b.v);
        }
        found = nn;
      } else { /* array -> bitmap (duplicates collapse) */
#pragma omp parallel for schedule(static)
        for (int64_t w = 0; w < words; ++w) fbm[w] = 0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < found; ++i)
          __atomic_fetch_or(&fbm[front[i] >> 6], 1ull << (front[i] & 63), __ATOMIC_RELAXED);
      }
      top_down = next_td;
    }
    nf = found;
  }
  *secs = now_s() - t0;
  if (entries) *entries = total_entries;
  free(front);
  free(next);
  free(fbm);
  free(nbm);
  free(vis);
  return levels;
}
