// Seeded synthetic graph generators and a symmetric CSR builder.
//
// This file produces INPUTS only.  It holds no breadth-first-search
// arithmetic: both the serial checker and the GPU library consume the CSR
// arrays built here, and neither shares any other code with this file.
//
// Graph families (shapes of the workloads the paper evaluates, Table 1):
//   * R-MAT / Kronecker-like power-law graphs (stand-in for kron_23 and the
//     small-diameter real-world graphs),
//   * uniform random graphs (stand-in for urand_25),
//   * a perturbed 2D lattice (stand-in for the large-diameter road / mesh /
//     kNN class).
//
// Every random number is a pure function of (seed, counter): the SplitMix64
// output function (Steele, Lea and Flood, OOPSLA 2014) evaluated at state
// seed + (counter + 1) * 0x9E3779B97F4A7C15.  Results therefore do not depend
// on the number of OpenMP threads.
//
// Output CSR invariants: row_ptr[0] = 0, row_ptr[n] = nnz, rows sorted
// ascending, no duplicates, no self-loops, symmetric (v in N(u) <=> u in N(v)).

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Element `ctr` of the SplitMix64 sequence started at state `seed`.
inline uint64_t draw(uint64_t seed, uint64_t ctr) {
  return splitmix_out(seed + (ctr + 1) * kGolden);
}

// Uniform integer in [0, bound) by the multiply-high method (Lemire 2019,
// without the rejection step; the bias is below 2^-40 for bound < 2^24).
inline uint64_t below(uint64_t r, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

struct Csr {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
};

void csr_free(Csr* g) {
  if (!g) return;
  std::free(g->row_ptr);
  std::free(g->col);
  delete g;
}

template <class T>
T* alloc_array(size_t count) {
  void* p = std::malloc(count ? count * sizeof(T) : sizeof(T));
  return static_cast<T*>(p);
}

// Exclusive prefix sum of `in[0..n)` into `out[0..n]` (out[n] = total),
// computed in parallel blocks so that large vertex counts stay fast.
void exclusive_scan(const int64_t* in, int64_t* out, int64_t n) {
  int nt = omp_get_max_threads();
  std::vector<int64_t> part(nt + 1, 0);
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int T = omp_get_num_threads();
    int64_t lo = n * t / T, hi = n * (t + 1) / T;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += in[i];
    part[t + 1] = s;
#pragma omp barrier
#pragma omp single
    for (int i = 1; i <= T; ++i) part[i] += part[i - 1];
    int64_t run = part[t];
    for (int64_t i = lo; i < hi; ++i) {
      out[i] = run;
      run += in[i];
    }
  }
  out[n] = part[nt];
}

// Builds a symmetric, deduplicated, self-loop-free CSR over `n` vertices from
// `m` undirected endpoint pairs.  Pairs with u == v are dropped; each kept
// pair contributes both directions; repeated pairs collapse to one entry.
Csr* build_symmetric(int64_t n, int64_t m, const int32_t* u, const int32_t* v) {
  Csr* g = new (std::nothrow) Csr;
  if (!g) return nullptr;
  g->n = n;
  int64_t* deg = alloc_array<int64_t>(n);
  int64_t* off = alloc_array<int64_t>(n + 1);
  if (!deg || !off) { std::free(deg); std::free(off); delete g; return nullptr; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg[i] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = u[e], b = v[e];
    if (a == b) continue;
    __atomic_fetch_add(&deg[a], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[b], 1, __ATOMIC_RELAXED);
  }
  exclusive_scan(deg, off, n);
  int64_t total = off[n];
  int32_t* tmp = alloc_array<int32_t>(total);
  if (!tmp) { std::free(deg); std::free(off); delete g; return nullptr; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg[i] = off[i];  // reuse as cursor
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = u[e], b = v[e];
    if (a == b) continue;
    int64_t pa = __atomic_fetch_add(&deg[a], 1, __ATOMIC_RELAXED);
    int64_t pb = __atomic_fetch_add(&deg[b], 1, __ATOMIC_RELAXED);
    tmp[pa] = b;
    tmp[pb] = a;
  }
  // Sort each row and drop repeats; deg[] now receives the unique count.
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; ++r) {
    int32_t* beg = tmp + off[r];
    int32_t* end = tmp + off[r + 1];
    std::sort(beg, end);
    deg[r] = std::unique(beg, end) - beg;
  }
  g->row_ptr = alloc_array<int64_t>(n + 1);
  if (!g->row_ptr) { std::free(tmp); std::free(deg); std::free(off); delete g; return nullptr; }
  exclusive_scan(deg, g->row_ptr, n);
  g->nnz = g->row_ptr[n];
  g->col = alloc_array<int32_t>(g->nnz);
  if (!g->col) { std::free(tmp); std::free(deg); std::free(off); csr_free(g); return nullptr; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t r = 0; r < n; ++r)
    std::memcpy(g->col + g->row_ptr[r], tmp + off[r], sizeof(int32_t) * deg[r]);
  std::free(tmp);
  std::free(deg);
  std::free(off);
  return g;
}

// Seeded uniform permutation of [0, n) (Fisher-Yates, serial so that the
// result is a function of the seed alone).
std::vector<int32_t> permutation(int64_t n, uint64_t seed) {
  std::vector<int32_t> p(n);
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t j = n - 1; j > 0; --j) {
    int64_t k = (int64_t)below(draw(seed, (uint64_t)j), (uint64_t)(j + 1));
    std::swap(p[j], p[k]);
  }
  return p;
}

}  // namespace

extern "C" {

void gg_free(void* h) { csr_free(static_cast<Csr*>(h)); }
int64_t gg_n(void* h) { return static_cast<Csr*>(h)->n; }
int64_t gg_nnz(void* h) { return static_cast<Csr*>(h)->nnz; }
int64_t* gg_row_ptr(void* h) { return static_cast<Csr*>(h)->row_ptr; }
int32_t* gg_col(void* h) { return static_cast<Csr*>(h)->col; }

uint64_t gg_draw(uint64_t seed, uint64_t ctr) { return draw(seed, ctr); }

// Symmetric CSR from caller-supplied endpoint pairs (ids in [0, n)).
void* gg_from_edges(int64_t n, int64_t m, const int32_t* u, const int32_t* v) {
  if (n < 1 || n > INT32_MAX || m < 0) return nullptr;
  for (int64_t e = 0; e < m; ++e)
    if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) return nullptr;
  return build_symmetric(n, m, u, v);
}

// R-MAT graph: 2^scale vertices, edge_factor * 2^scale sampled pairs.  Each
// sample descends `scale` quadrant choices with probabilities (a, b, c,
// 1-a-b-c) for (top-left, top-right, bottom-left, bottom-right), no noise.
// Vertex ids are then relabelled through a seeded permutation.
void* gg_rmat(int scale, int edge_factor, double a, double b, double c,
              uint64_t seed, uint64_t perm_seed) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return nullptr;
  int64_t n = (int64_t)1 << scale;
  int64_t m = (int64_t)edge_factor * n;
  const double two32 = 4294967296.0;
  const uint64_t ta = (uint64_t)(a * two32);
  const uint64_t tab = (uint64_t)((a + b) * two32);
  const uint64_t tabc = (uint64_t)((a + b + c) * two32);
  std::vector<int32_t> perm = permutation(n, perm_seed);
  int32_t* u = alloc_array<int32_t>(m);
  int32_t* v = alloc_array<int32_t>(m);
  if (!u || !v) { std::free(u); std::free(v); return nullptr; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t r = 0, col = 0;
    uint64_t word = 0;
    for (int l = 0; l < scale; ++l) {
      if ((l & 1) == 0) word = draw(seed, (uint64_t)i * 16 + (uint64_t)(l >> 1));
      uint64_t x = (l & 1) ? (word >> 32) : (word & 0xFFFFFFFFull);
      uint32_t bu, bv;
      if (x < ta) { bu = 0; bv = 0; }
      else if (x < tab) { bu = 0; bv = 1; }
      else if (x < tabc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      r = (r << 1) | bu;
      col = (col << 1) | bv;
    }
    u[i] = perm[r];
    v[i] = perm[col];
  }
  Csr* g = build_symmetric(n, m, u, v);
  std::free(u);
  std::free(v);
  return g;
}

// Uniform random graph: n vertices, n * avg_degree / 2 uniformly drawn
// endpoint pairs, then symmetrised and deduplicated.
void* gg_urand(int64_t n, int avg_degree, uint64_t seed) {
  if (n < 2 || n > INT32_MAX || avg_degree < 1) return nullptr;
  int64_t m = n * avg_degree / 2;
  int32_t* u = alloc_array<int32_t>(m);
  int32_t* v = alloc_array<int32_t>(m);
  if (!u || !v) { std::free(u); std::free(v); return nullptr; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    u[i] = (int32_t)below(draw(seed, 2 * (uint64_t)i), (uint64_t)n);
    v[i] = (int32_t)below(draw(seed, 2 * (uint64_t)i + 1), (uint64_t)n);
  }
  Csr* g = build_symmetric(n, m, u, v);
  std::free(u);
  std::free(v);
  return g;
}

// Perturbed 2D lattice.  Vertex (r, c) has id r * width + c (no relabelling,
// so mesh locality is kept).  Each of the 2 * width * (width - 1) lattice
// edges is kept independently with probability 1 - p_delete.  Then exactly
// floor(p_shortcut * n) distinct vertices, chosen by a seeded partial
// shuffle, each receive one extra edge to a vertex drawn uniformly among the
// in-grid vertices at Manhattan distance 1..radius (a shortcut that lands on
// an existing edge collapses in deduplication).
void* gg_grid(int64_t width, double p_delete, double p_shortcut, int radius, uint64_t seed) {
  if (width < 2 || width * width > INT32_MAX || radius < 0) return nullptr;
  const int64_t n = width * width;
  const int64_t nh = width * (width - 1);  // horizontal edges, then vertical
  const int64_t lattice = 2 * nh;
  const uint64_t del_seed = draw(seed, 0x6401);
  const uint64_t sel_seed = draw(seed, 0x6402);
  const uint64_t tgt_seed = draw(seed, 0x6403);
  const double two64 = 18446744073709551616.0;
  const uint64_t keep_below = p_delete <= 0 ? UINT64_MAX : (uint64_t)((1.0 - p_delete) * two64);
  const int64_t n_short = (int64_t)(p_shortcut * (double)n);
  int32_t* u = alloc_array<int32_t>(lattice + n_short);
  int32_t* v = alloc_array<int32_t>(lattice + n_short);
  if (!u || !v) { std::free(u); std::free(v); return nullptr; }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < lattice; ++e) {
    int64_t a, b;
    if (e < nh) {
      int64_t r = e / (width - 1), c = e % (width - 1);
      a = r * width + c; b = a + 1;
    } else {
      int64_t k = e - nh;
      int64_t r = k / width, c = k % width;
      a = r * width + c; b = a + width;
    }
    bool keep = p_delete <= 0 || draw(del_seed, (uint64_t)e) < keep_below;
    u[e] = (int32_t)a;
    v[e] = keep ? (int32_t)b : (int32_t)a;  // a dropped edge becomes a self-loop, removed later
  }
  if (n_short > 0) {
    // Partial Fisher-Yates: the first n_short slots are a uniform sample of
    // distinct vertices.
    std::vector<int32_t> pool(n);
    for (int64_t i = 0; i < n; ++i) pool[i] = (int32_t)i;
    for (int64_t j = 0; j < n_short; ++j) {
      int64_t k = j + (int64_t)below(draw(sel_seed, (uint64_t)j), (uint64_t)(n - j));
      std::swap(pool[j], pool[k]);
    }
    // Offsets (dr, dc) with 1 <= |dr| + |dc| <= radius.
    std::vector<std::pair<int, int>> offs;
    for (int dr = -radius; dr <= radius; ++dr)
      for (int dc = -radius; dc <= radius; ++dc) {
        int d = std::abs(dr) + std::abs(dc);
        if (d >= 1 && d <= radius) offs.emplace_back(dr, dc);
      }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_short; ++j) {
      int64_t s = pool[j];
      int64_t r = s / width, c = s % width;
      int cnt = 0;
      for (auto& o : offs) {
        int64_t rr = r + o.first, cc = c + o.second;
        if (rr >= 0 && rr < width && cc >= 0 && cc < width) ++cnt;
      }
      int64_t pick = cnt ? (int64_t)below(draw(tgt_seed, (uint64_t)j), (uint64_t)cnt) : -1;
      int64_t t = s;
      for (auto& o : offs) {
        int64_t rr = r + o.first, cc = c + o.second;
        if (rr >= 0 && rr < width && cc >= 0 && cc < width) {
          if (pick-- == 0) { t = rr * width + cc; break; }
        }
      }
      u[lattice + j] = (int32_t)s;
      v[lattice + j] = (int32_t)t;
    }
  }
  Csr* g = build_symmetric(n, lattice + n_short, u, v);
  std::free(u);
  std::free(v);
  return g;
}

// Draws up to k distinct vertices with nonzero degree, uniformly, from the
// seed.  Returns the number written (fewer than k only when the graph has
// fewer than k non-isolated vertices).
int64_t gg_sources(int64_t n, const int64_t* row_ptr, int64_t k, uint64_t seed, int32_t* out) {
  int64_t nonisolated = 0;
  for (int64_t i = 0; i < n; ++i) nonisolated += row_ptr[i + 1] > row_ptr[i];
  int64_t want = std::min<int64_t>(k, nonisolated);
  std::vector<char> taken(n, 0);
  int64_t got = 0;
  for (uint64_t ctr = 0; got < want; ++ctr) {
    int64_t c = (int64_t)below(draw(seed, ctr), (uint64_t)n);
    if (row_ptr[c + 1] > row_ptr[c] && !taken[c]) {
      taken[c] = 1;
      out[got++] = (int32_t)c;
    }
  }
  return got;
}

}  // extern "C"
