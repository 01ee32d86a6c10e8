// Single-source direction-optimizing BFS on gfx950.
//
// The search is level-synchronous (Section 2, Listing 1): level L expands
// the vertices at distance L and discovers those at distance L + 1.  Each
// level runs in one of two directions (Section 2, BFS-Hybrid):
//   top-down  - every frontier vertex examines its neighbours; a neighbour
//               whose visited bit is clear is claimed with one atomicOr on
//               its visited word, and the winner stores dist and parent
//               with plain stores (Section 2, BFS-NonAtomic: no atomic on
//               the distance) and appends the vertex to the next frontier
//               queue;
//   bottom-up - every unvisited vertex scans its own row for a neighbour in
//               the frontier bitmap and stops at the first hit (Section 2,
//               Listing 2).
// Visited state lives in a bitmap (Section 2, BFS-VisitedBitmap).  A bit of
// a packed bitmap is never set with a plain read-modify-write from two
// threads: top-down uses atomicOr, bottom-up gives each 64-vertex word to
// one wavefront, which alone writes it.  (For the paper's ablation the
// top-down claim can instead be a compare-and-swap on the distance or a
// plain test and store: bfs_params.td_visited.)
//
// Mapping onto CDNA4 (wave64), one kernel launch per level (k_level):
//   * top-down work is split by degree into roles of one launch: a thread
//     per vertex of degree <= t1, a wavefront (or, for few long rows,
//     several) per vertex of degree in (t1, t2], a workgroup per t2-edge
//     chunk of larger vertices; discoveries are staged in LDS per degree
//     class (ballot + mbcnt slots) and copied out with one global atomicAdd
//     per workgroup and class;
//   * bottom-up gives each wavefront a run of 64 visited words, compacts
//     their unvisited vertices into batches of 64 candidates, tests the
//     first neighbours from a 16-byte head record per vertex and scans the
//     rest of the rows that miss 64 at a time; the found masks become the
//     next-frontier and visited words with one coalesced store per run;
//   * hybrid searches keep the frontier bitmap exact during top-down levels
//     (set on discovery, cleared on expansion), and the top-down level after
//     a bottom-up phase reads its frontier from that bitmap, so no level
//     converts between queue and bitmap form;
//   * the level's counts are reduced by the level kernel itself: the last
//     workgroup to arrive applies the direction rule (Section 2: alpha/beta
//     of BFS-Hybrid dagger, or the 5 % frontier rule of BFS-Hybrid; Section
//     3: top-down only below average degree 7) and advances the control
//     block.
// Every kernel reads the level state from the control block, so the same
// kernel serves a host-driven loop, a queued loop and a captured hipGraph of
// many levels; each launch checks that the level it reads is the one it was
// made for.

#include <algorithm>
#include <chrono>
#include <cstring>

#include "common.h"
#include "device_util.h"

namespace bfsmi {
namespace {

// Writes the workgroup totals of K per-thread counters to this workgroup's
// slot of the partials array (plain stores; the decide step reduces them).
// Every thread of the workgroup must call it.
template <int K, class RowT>
__device__ __forceinline__ void block_partials(const DevG<RowT> &G, const unsigned long long (&v)[K],
                                               unsigned slot = blockIdx.x) {
  __shared__ unsigned long long part[K][16];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    unsigned long long s = wave_sum(v[k]);
    if (lane_id() == 0) part[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    unsigned long long t = 0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += part[threadIdx.x][i];
    G.partials[(size_t)slot * kPartials + threadIdx.x] = t;
  }
}

// Marks the running level as having lost queue entries (an append past a
// queue's end).  Any thread; the decide step reads the flag.
__device__ __forceinline__ void flag_overflow(Ctl *c) {
  __hip_atomic_fetch_or(&c->overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claims vertex v: true for exactly one caller per search.
__device__ __forceinline__ bool claim(uint64_t *vis, int32_t v) {
  const uint64_t bit = 1ull << (v & 63);
  unsigned long long *w = reinterpret_cast<unsigned long long *>(vis + (v >> 6));
  if (*w & bit) return false;  // already visited (a stale read only costs the atomic below)
  return !(atomicOr(w, (unsigned long long)bit) & bit);
}

template <class RowT>
__device__ __forceinline__ int bucket_of(const DevG<RowT> &G, int64_t deg) {
  return deg <= G.t1 ? kSmall : (deg <= G.t2 ? kMedium : kLarge);
}

// Workgroup staging of discovered vertices in LDS, one buffer per degree
// class.  Lanes reserve slots with LDS atomics; the workgroup copies the
// buffers out with one global atomicAdd per class whenever they are half
// full (at workgroup-uniform points) and at the end.  Slots past a buffer's
// capacity go straight to the global queue.  Layout of the dynamic LDS:
// counts[4] | small[8 * bs] | medium[2 * bs] | large[bs] (8-byte entries).
// Large vertices are queued one entry each, {chunk count, vertex}, and the
// queue set's chunk total is kept beside its counts: the top-down level that
// expands them maps its chunk indices onto the entries (wv / wp: one window
// of entries and the inclusive prefix sums of their chunk counts).  A hub's
// chunks are thus never written out when the next level runs bottom-up.
// Capacities per thread of the workgroup: 8 small, 4 medium, 2 large (a
// large-role step claims two neighbours per thread, so with a flush after
// each step its medium and large discoveries always fit: a hub-first row's
// first chunk finds mostly hubs).
struct Stage {
  unsigned *cnt;
  int32_t *small;
  int32_t *medium;
  uint64_t *large;
  uint64_t *wv;
  unsigned *wp;
  unsigned cap_small, cap_medium, cap_large;
  // (8, 4 and 2 entries per thread: computed, not looked up, so that a
  // thread-dependent class does not put the struct in scratch memory)
  __device__ unsigned cap(int b) const { return (8u * blockDim.x) >> b; }
};

__host__ __device__ constexpr size_t stage_bytes(int bs) { return 16 + (size_t)76 * bs; }

__device__ __forceinline__ Stage stage_open(char *lds) {
  const unsigned bs = blockDim.x;
  Stage S;
  S.cnt = reinterpret_cast<unsigned *>(lds);
  S.small = reinterpret_cast<int32_t *>(lds + 16);
  S.medium = S.small + 8 * bs;
  S.large = reinterpret_cast<uint64_t *>(S.medium + 4 * bs);
  S.wv = S.large + 2 * bs;
  S.wp = reinterpret_cast<unsigned *>(S.wv + bs);
  S.cap_small = 8 * bs;
  S.cap_medium = 4 * bs;
  S.cap_large = 2 * bs;
  if (threadIdx.x < 3) S.cnt[threadIdx.x] = 0;
  __syncthreads();
  return S;
}

template <class RowT>
__device__ __forceinline__ int32_t *global_queue(const DevG<RowT> &G, int qn, int b) {
  return b == kSmall ? (qn ? G.qs[1] : G.qs[0]) : (qn ? G.qm[1] : G.qm[0]);
}

// Appends the lanes' discovered vertices (queue set `qn`), split by degree
// class.  Must be called by all lanes of a wavefront together.
template <class RowT>
__device__ __forceinline__ void wave_stage(const DevG<RowT> &G, const Stage &S, int qn, bool found,
                                           int32_t v, int64_t deg) {
  const int b = found ? bucket_of(G, deg) : -1;
  const int lane = lane_id();
#pragma unroll
  for (int bb = kSmall; bb <= kMedium; ++bb) {
    const uint64_t m = __ballot(b == bb);
    if (!m) continue;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const unsigned k = (unsigned)__popcll(m);
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&S.cnt[bb], k);
    base = __shfl(base, leader);
    const unsigned cap = S.cap(bb);
    const unsigned first_over = base > cap ? base : cap;
    const unsigned over = base + k > cap ? base + k - first_over : 0;
    unsigned gbase = 0;
    if (over) {
      if (lane == leader) gbase = atomicAdd(&G.ctl->qcnt[qn][bb], over);
      gbase = __shfl(gbase, leader);
    }
    if (b == bb) {
      const unsigned slot = base + lanes_below(m);
      if (slot < cap)
        (bb == kSmall ? S.small : S.medium)[slot] = v;
      else if (gbase + (slot - first_over) < G.qcap && gbase + (slot - first_over) >= gbase) {
        st_x(global_queue(G, qn, bb) + gbase + (slot - first_over), v, G.pers);
        if (G.slot) st_x(G.slot + v, (int32_t)(gbase + (slot - first_over)), G.pers);
      } else {
        flag_overflow(G.ctl);  // past the end: dropped, and the decide step stops the search
      }
    }
  }
  // Large vertices (rare): one staged entry each, {chunk count, vertex}.
  // Lanes past the buffer append theirs at once (one reservation for the
  // wavefront's spilled entries, and their chunks added to the set's total).
  const bool isl = b == kLarge;
  const uint64_t lm = __ballot(isl);
  if (lm) {
    const int leader = __ffsll((unsigned long long)lm) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&S.cnt[kLarge], (unsigned)__popcll(lm));
    base = __shfl(base, leader);
    const unsigned nch = isl ? (unsigned)((deg + G.t2 - 1) / G.t2) : 0u;
    const uint64_t ent = ((uint64_t)nch << 32) | (uint32_t)v;
    const unsigned slot = base + lanes_below(lm);
    if (isl && slot < S.cap_large) S.large[slot] = ent;
    const bool spill = isl && slot >= S.cap_large;
    const uint64_t om = __ballot(spill);
    if (om) {
      const int sl = __ffsll((unsigned long long)om) - 1;
      const unsigned long long chunks = wave_sum(spill ? (unsigned long long)nch : 0ull);
      unsigned gbase = 0;
      if (lane == sl) {
        gbase = atomicAdd(&G.ctl->qcnt[qn][kLarge], (unsigned)__popcll(om));
        atomicAdd(&G.ctl->qchunk[qn], (unsigned)chunks);
      }
      gbase = __shfl(gbase, sl);
      if (spill) {
        const uint64_t pos = (uint64_t)gbase + lanes_below(om);
        if (pos < G.lcap)
          st_x((qn ? G.ql[1] : G.ql[0]) + pos, ent, G.pers);
        else
          flag_overflow(G.ctl);  // past the end: dropped, and the decide step stops the search
      }
    }
  }
}

// Inclusive prefix sum of x over the threads of the workgroup (thread
// order).  Every thread of the workgroup calls it.
__device__ __forceinline__ unsigned block_incl_scan(unsigned x) {
  __shared__ unsigned wtot[16];
  const int lane = lane_id(), w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  if (lane == kWave - 1) wtot[w] = x;
  __syncthreads();
  unsigned before = 0;
  for (int i = 0; i < w; ++i) before += wtot[i];
  __syncthreads();  // (wtot is reused by the next call)
  return x + before;
}

// Copies the staged entries to queue set `qn` and empties the buffers; with
// `only_if_half_full`, only when some buffer is at least half full.  All
// threads of the workgroup call it at the same point.
template <class RowT>
__device__ __forceinline__ void stage_flush(const DevG<RowT> &G, const Stage &S, int qn,
                                            bool only_if_half_full = false) {
  __shared__ unsigned gbase[3], count[3], lchunks;
  __syncthreads();
  const unsigned bs = blockDim.x;
  if (only_if_half_full) {
    const bool skip = S.cnt[kSmall] < 4 * bs && S.cnt[kMedium] < 2 * bs && S.cnt[kLarge] < bs;
    // every thread has read the counts before any wavefront can stage again
    __syncthreads();
    if (skip) return;  // uniform: the same counts were read by every thread
  }
  // the staged large vertices' chunks, summed (entries 2t and 2t + 1 are
  // thread t's: at most 2 bs staged)
  {
    const unsigned nl = S.cnt[kLarge] < S.cap_large ? S.cnt[kLarge] : S.cap_large;
    const unsigned i0 = 2 * threadIdx.x, i1 = i0 + 1;
    const unsigned c0 = i0 < nl ? (unsigned)(S.large[i0] >> 32) : 0u;
    const unsigned c1 = i1 < nl ? (unsigned)(S.large[i1] >> 32) : 0u;
    const unsigned incl = block_incl_scan(c0 + c1);
    if (threadIdx.x == bs - 1) lchunks = incl;
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    const unsigned b = threadIdx.x;
    const unsigned n = S.cnt[b] < S.cap(b) ? S.cnt[b] : S.cap(b);
    count[b] = n;
    gbase[b] = n ? atomicAdd(&G.ctl->qcnt[qn][b], n) : 0;
    if (b == kLarge && n) atomicAdd(&G.ctl->qchunk[qn], lchunks);
    // a range past the queue's end (or past 2^32 appends) loses entries: the
    // search stops at this level's decide step
    const uint64_t qend = (uint64_t)gbase[b] + n;
    if (n && qend > (b == kLarge ? G.lcap : G.qcap)) flag_overflow(G.ctl);
  }
  __syncthreads();
  int32_t *qs = global_queue(G, qn, kSmall);
  int32_t *qm = global_queue(G, qn, kMedium);
  uint64_t *ql = qn ? G.ql[1] : G.ql[0];
  // entries that would land past a queue's end are dropped (the counts still
  // grow, and the decide step turns that into an error)
  for (unsigned i = threadIdx.x; i < count[kSmall]; i += blockDim.x)
    if (gbase[kSmall] + i < G.qcap) {
      st_x(qs + gbase[kSmall] + i, S.small[i], G.pers);
      if (G.slot) st_x(G.slot + S.small[i], (int32_t)(gbase[kSmall] + i), G.pers);
    }
  for (unsigned i = threadIdx.x; i < count[kMedium]; i += blockDim.x)
    if (gbase[kMedium] + i < G.qcap) {
      st_x(qm + gbase[kMedium] + i, S.medium[i], G.pers);
      if (G.slot) st_x(G.slot + S.medium[i], (int32_t)(gbase[kMedium] + i), G.pers);
    }
  for (unsigned i = threadIdx.x; i < count[kLarge]; i += blockDim.x)
    if (gbase[kLarge] + i < G.lcap) st_x(ql + gbase[kLarge] + i, S.large[i], G.pers);
  __syncthreads();
  if (threadIdx.x < 3) S.cnt[threadIdx.x] = 0;
  __syncthreads();
}

// Copies the control block to its host-mapped mirror, then bumps the
// mirror's sequence number (system-scope release), so a host thread polling
// that number sees a complete level state.  One thread.
__device__ void publish(Ctl *c) {
  Ctl *m = c->mirror;
  if (!m) return;
  const uint32_t seq = c->seq + 1;
  c->seq = seq;
  __hip_atomic_store(&m->seq_wip, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
  const uint64_t *src = reinterpret_cast<const uint64_t *>(c);
  uint64_t *dst = reinterpret_cast<uint64_t *>(m);
  constexpr int kWords = (int)(offsetof(Ctl, seq) / sizeof(uint64_t));
  for (int i = 0; i < kWords; ++i) dst[i] = src[i];
  __threadfence_system();
  __hip_atomic_store(&m->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// Initialisation: dist = -1, parent = -1, visited = isolated-vertex mask,
// both frontier bitmaps and the partial counts cleared, then the source at
// level 0 in queue set 0
// (the first level is top-down).

// a[0, n) = -1 except a[s] = sv, with streaming stores: 4-byte stores up to
// the first 16-byte boundary and past the last, 16-byte stores between.
__device__ __forceinline__ void init_fill(int32_t *a, int64_t n, int32_t s, int32_t sv, int64_t tid,
                                          int64_t stride) {
  typedef int32_t v4i __attribute__((ext_vector_type(4)));
  const int64_t head = min(n, (int64_t)(((16u - (reinterpret_cast<uintptr_t>(a) & 15u)) & 15u) >> 2));
  const int64_t groups = (n - head) >> 2;
  for (int64_t i = tid; i < head; i += stride) __builtin_nontemporal_store(i == s ? sv : -1, gptr(a + i));
  v4i *a4 = reinterpret_cast<v4i *>(a + head);
  for (int64_t q = tid; q < groups; q += stride) {
    const int64_t i0 = head + 4 * q;
    v4i x = {-1, -1, -1, -1};
    if (s >= i0 && s < i0 + 4) x[s - i0] = sv;
    __builtin_nontemporal_store(x, a4 + q);
  }
  for (int64_t i = head + 4 * groups + tid; i < n; i += stride)
    __builtin_nontemporal_store(i == s ? sv : -1, gptr(a + i));
}

template <class RowT>
__global__ void k_init(DevG<RowT> G, int32_t s, int32_t *dist, int32_t *parent, int32_t policy,
                       int32_t alpha, int32_t beta, int64_t nnz, int32_t rec_cap, Ctl *mirror,
                       uint32_t seq0, int32_t pub_mode) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // streaming stores: left dirty in the caches, these lines would be written
  // back during the first dense level and slow it (-5 % per search); 16
  // bytes a lane over the 16-byte-aligned middle of each array
  init_fill(dist, G.n, s, 0, tid, stride);
  if (parent) init_fill(parent, G.n, s, s, tid, stride);
  const int64_t sw = s >> 6;
  const uint64_t sb = 1ull << (s & 63);
  for (int64_t w = tid; w < G.words; w += stride) {
    G.vis[w] = G.iso[w] | (w == sw ? sb : 0ull);
    // hybrid searches keep bm[0] as the current frontier bitmap from level 0
    G.bm[0][w] = (policy != BFS_POLICY_TD_ONLY && w == sw) ? sb : 0ull;
    G.bm[1][w] = 0;
  }
  if (G.sshift >= 0) {  // summaries: bm[0]'s holds the source's word
    const int64_t sb = sw >> G.sshift;
    for (int64_t w = tid; w < G.swords; w += stride) {
      G.sm[0][w] = (policy != BFS_POLICY_TD_ONLY && w == (sb >> 6)) ? 1ull << (sb & 63) : 0ull;
      G.sm[1][w] = 0;
    }
  }
  for (int64_t i = tid; i < (int64_t)kPartialsAlloc; i += stride) G.partials[i] = 0;  // and arrivals
  if (tid == 0) {
    Ctl *c = G.ctl;
    const int64_t deg = (int64_t)G.rp[s + 1] - (int64_t)G.rp[s];
    c->level = 0;
    c->dir = kTD;
    c->done = 0;
    c->qcur = 0;
    c->bcur = 0;
    c->conv = kConvNone;
    c->policy = policy;
    c->alpha = alpha;
    c->beta = beta;
    c->rec_cap = rec_cap;
    c->levels_done = 0;
    c->overflow = 0;
    c->qcap[0] = G.qcap;
    c->qcap[1] = G.lcap;
    c->n = G.n;
    c->nnz = nnz;
    c->n_f = 1;
    // (classless searches add a level's m_f up while expanding it)
    c->classless = G.classless;
    c->sum_ok[0] = 1;
    c->sum_ok[1] = 1;
    c->m_f = G.classless ? 0 : deg;
    c->m_u = G.classless ? nnz : nnz - deg;
    c->sum_mf = 0;
    c->reached = 1;
    for (int q = 0; q < 2; ++q) {
      for (int b = 0; b < 3; ++b) c->qcnt[q][b] = 0;
      c->qchunk[q] = 0;
    }
    const int b = bucket_of(G, deg);
    if (b == kLarge) {
      const unsigned nch = (unsigned)((deg + G.t2 - 1) / G.t2);
      G.ql[0][0] = ((uint64_t)nch << 32) | (uint32_t)s;
      c->qcnt[0][kLarge] = 1;
      c->qchunk[0] = nch;
    } else {
      (b == kSmall ? G.qs[0] : G.qm[0])[0] = s;
      if (G.slot) G.slot[s] = 0;
      c->qcnt[0][b] = 1;
    }
    c->dist = dist;
    c->parent = parent;
    c->pub_mode = pub_mode;
    c->mirror = mirror;
    c->bar_count = 0;
    c->bar_gen = 0;
    c->seq = seq0;  // publication numbers continue across runs, so a stale
    publish(c);     // mirror never matches the number a new run waits for
  }
}

// A bottom-up level copies the frontier summary into LDS when the frontier
// has at most this many vertices per bitmap word.
constexpr int64_t kSumFrontierWords = 2;

// A top-down level keeps the occupancy summary of the frontier bitmap only
// while the frontier it makes could be small enough for a bottom-up level to
// test the summary.  Its expected size is the level's edges times the share
// of edge ends not yet visited, m_f * m_u / nnz; where that is more than
// twice the bottom-up level's limit, the level skips the summary's atomics
// (on a hub-heavy level a third of its memory-side atomics), and the
// summary counts as incomplete until a bottom-up level has rewritten it.
// The top-down level and the decide step evaluate this with the same
// values (the control block's m_f and m_u before the decide step).
__host__ __device__ inline bool td_keeps_summary(int64_t m_f, int64_t m_u, int64_t n, int64_t nnz) {
  return (double)m_f * (double)m_u <= (double)(2 * kSumFrontierWords) * (double)((n + 63) >> 6) * (double)nnz;
}

// Moves the control block's level number on with an agent-scope atomic
// exchange and waits for it to return, i.e. until it has been performed at
// the device-wide coherence point.  A plain store would sit in this XCD's L2
// (written back only at a release or at the kernel's end), where a workgroup
// on another XCD, which reads the number with an agent-scope load, need not
// see it.  One thread.
__device__ __forceinline__ void publish_level(Ctl *c, int32_t level) {
  (void)__hip_atomic_exchange(&c->level, level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Level bookkeeping and the direction rule, applied by one thread to the
// level's totals {found, degree sum of found, scanned, examined}.
// `bumped` >= 0: the caller has already stored level bumped + 1 and waited
// for that store (it overlapped the caller's last round trip).
__device__ void decide_apply(Ctl *c, LevelRec *recs, const unsigned long long (&tot)[kPartials],
                             int32_t bumped = -1) {
  const int32_t L = bumped >= 0 ? bumped : c->level;
  const int32_t cur = c->dir;
  // The level number changes first, and has been performed at device scope
  // before any other field changes: a workgroup of this level's launch that
  // starts only now reads the fields, then the number, and leaves when the
  // number moved on (see publish_level).
  if (bumped < 0) publish_level(c, L + 1);
  const int64_t found = (int64_t)tot[0];
  // tot[1]: the degree sum of the vertices found, i.e. the next level's m_f;
  // in a classless search, this level's own m_f (summed while expanding)
  const bool classless = c->classless != 0;
  const int64_t fdeg = classless ? 0 : (int64_t)tot[1];
  const int64_t mf = classless ? (int64_t)tot[1] : c->m_f;
  if (classless) c->m_u -= mf;
  if (L < c->rec_cap) {
    LevelRec r;
    r.level = L;
    r.dir = cur;
    r.n_f = c->n_f;
    r.m_f = mf;
    r.m_u = c->m_u;
    r.found = found;
    r.scanned = (int64_t)tot[2];
    r.examined = (int64_t)tot[3];
    recs[L] = r;
  }
  c->levels_done = L + 1;
  c->sum_mf += mf;
  c->reached += found;
  if (cur == kTD) {
    // the next frontier was appended to the other queue set; the old set
    // becomes the target of the following top-down level
    for (int b = 0; b < 3; ++b) c->qcnt[c->qcur][b] = 0;
    c->qchunk[c->qcur] = 0;
    c->qcur ^= 1;
    if (!td_keeps_summary(mf, c->m_u, c->n, c->nnz)) c->sum_ok[c->bcur] = 0;  // it skipped its summary bits
    // with the visited test of plain loads and stores a vertex can be
    // appended once per racing discoverer; a set that outgrew its queues
    // lost entries, so the search ends here and the host reports it
    const unsigned *q = c->qcnt[c->qcur];
    if (__hip_atomic_load(&c->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
        q[kSmall] > c->qcap[0] || q[kMedium] > c->qcap[0] || q[kLarge] > c->qcap[1]) {
      c->overflow = 1;
      c->done = 1;
      c->conv = kConvNone;
      publish(c);
      return;
    }
  } else {
    c->bcur ^= 1;
    c->sum_ok[c->bcur] = 1;  // written whole by the level (read only where it was)
  }
  if (found == 0) {
    c->done = 1;
    c->conv = kConvNone;
    publish(c);
    return;
  }
  const int64_t m_u = c->m_u - fdeg;
  int32_t nxt;
  if (c->policy == BFS_POLICY_TD_ONLY) {
    nxt = kTD;
  } else if (c->policy == BFS_POLICY_FRONTIER_5PCT) {
    nxt = (20 * found >= c->n) ? kBU : kTD;
  } else if (cur == kTD) {
    nxt = (fdeg * (int64_t)c->alpha > m_u) ? kBU : kTD;
  } else {
    nxt = (found * (int64_t)c->beta < c->n && found < c->n_f) ? kTD : kBU;
  }
  // (top-down levels keep the frontier bitmap of hybrid searches current, so
  // only a switch back to top-down changes how the frontier is read)
  c->conv = (cur == kBU && nxt == kTD) ? kConvB2Q : kConvNone;
  if (c->conv == kConvB2Q) {
    for (int b = 0; b < 3; ++b) c->qcnt[c->qcur][b] = 0;
    c->qchunk[c->qcur] = 0;
  }
  c->n_f = found;
  c->m_f = fdeg;
  c->m_u = m_u;
  c->dir = nxt;
  if (c->pub_mode == kPubEvery) publish(c);
}

// Reduces (and clears) the partial counts of `nblocks` workgroups; every
// thread of the calling workgroup takes part, thread 0 receives the totals.
// `same_kernel`: the partials were written by other workgroups of the
// running kernel (read them with device-scope atomics); otherwise by an
// earlier kernel (plain loads suffice).
template <bool same_kernel>
__device__ void reduce_partials(unsigned long long *partials, int nblocks, unsigned long long (&tot)[kPartials]) {
  __shared__ unsigned long long red[kPartials][16];
  unsigned long long v[kPartials] = {0, 0, 0, 0};
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kPartials; ++k) {
      unsigned long long *p = partials + (size_t)i * kPartials + k;
      if (same_kernel) {
        v[k] += __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        v[k] += *p;
        *p = 0;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kPartials; ++k) {
    const unsigned long long s = wave_sum(v[k]);
    if (lane_id() == 0) red[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < kPartials; ++k) tot[k] = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
      for (int k = 0; k < kPartials; ++k) tot[k] += red[k][w];
  }
}

// Discovery step shared by the top-down roles: the lane examines edge
// target v of frontier vertex u (when `has`), then the wavefront stages.
// Hybrid searches keep the current frontier bitmap exact through top-down
// levels: an expanded vertex leaves it, a discovered one enters it (the two
// sets are disjoint, and atomics on shared words commute), so a switch to
// bottom-up needs no conversion.  `fbm` is null for top-down-only searches.
// A vertex entering the bitmap also sets its word's bit in the bitmap's
// occupancy summary (`fsm`, null when the graph has none); bits leaving the
// bitmap leave the summary as it is, so it stays a superset of the occupied
// words until a bottom-up level rewrites it exactly.
__device__ __forceinline__ void fbm_set(uint64_t *fbm, uint64_t *fsm, int32_t sshift, int32_t v) {
  if (fbm) {
    atomicOr(reinterpret_cast<unsigned long long *>(fbm + (v >> 6)), 1ull << (v & 63));
    if (fsm) {
      const uint32_t sb = ((uint32_t)v >> 6) >> sshift;
      atomicOr(reinterpret_cast<unsigned long long *>(fsm + (sb >> 6)), 1ull << (sb & 63));
    }
  }
}
__device__ __forceinline__ void fbm_clear(uint64_t *fbm, int32_t u) {
  if (fbm) atomicAnd(reinterpret_cast<unsigned long long *>(fbm + (u >> 6)), ~(1ull << (u & 63)));
}

// Level state a top-down level needs, read once per level.
struct TdLevel {
  int32_t qcur, level;
  int64_t cnt[3];      // queue entries per class (large: one per vertex)
  int64_t nchunk;      // td_block_degree-edge chunks of the large vertices
  int64_t m_f;         // degree sum of the frontier (steers the medium-row split)
  int32_t *dist, *parent;
  uint64_t *fbm;       // current frontier bitmap (hybrid searches), else null
  uint64_t *fsm;       // its occupancy summary (null: none)
  int32_t sshift;      // bitmap words per summary bit, log2
  bool from_bitmap;    // the frontier is the bitmap of a bottom-up level
};

// The distance a top-down claim writes, and the distance read of the plain
// visited test.  Distances are streamed out (nothing reads them back), except
// that the plain test reads them: in the persistent kernel, where no kernel
// boundary separates the levels, those go through the device-coherent level
// (a store is complete before its workgroup arrives at the level's end).
template <class RowT>
__device__ __forceinline__ void dist_store(const DevG<RowT> &G, int32_t *p, int32_t d) {
  if (G.pers && G.td_visited != BFS_TD_VISITED_BITMAP && G.td_visited != BFS_TD_DIST_CAS)
    __hip_atomic_store(p, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    __builtin_nontemporal_store(d, gptr(p));
}
template <class RowT>
__device__ __forceinline__ int32_t dist_test_load(const DevG<RowT> &G, const int32_t *p) {
  return G.pers ? __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *gptr(p);
}

// Levels whose frontier has fewer edges than this claim with the atomic
// alone: reading the visited word first saves the atomics on vertices
// already visited, which only pays where there are many; on small levels
// it is one more dependent round trip (the lattice's levels: -5 %).
constexpr int64_t kPreloadMinEdges = 65536;

template <class RowT>
__device__ __forceinline__ void td_visit(const DevG<RowT> &G, const Stage &S, int qn, const TdLevel &T,
                                         bool has, int32_t u, int32_t v, bool preload,
                                         unsigned long long &nfound, unsigned long long &dfound) {
  const int32_t level = T.level;
  int32_t *dist = T.dist;
  int32_t *parent = T.parent;
  bool win = false;
  int64_t deg = 0;
  bool claimed = false;
  if (has) {
    if (G.td_visited == BFS_TD_VISITED_BITMAP) {
      if (preload) {
        claimed = claim(G.vis, v);
      } else {
        const uint64_t bit = 1ull << (v & 63);
        claimed = !(atomicOr(reinterpret_cast<unsigned long long *>(G.vis + (v >> 6)), (unsigned long long)bit) & bit);
      }
    }
    else if (G.td_visited == BFS_TD_DIST_CAS) claimed = atomicCAS(dist + v, -1, level + 1) == -1;
    else claimed = dist_test_load(G, dist + v) < 0;  // plain test: racing discoverers may all pass
  }
  if (claimed) {
    win = true;
    // (streaming stores, plain: every writer of v stores this same value)
    dist_store(G, dist + v, level + 1);
    if (parent) __builtin_nontemporal_store(u, gptr(parent + v));
    fbm_set(T.fbm, T.fsm, T.sshift, v);
    deg = G.classless ? 0 : G.head[v].x;
    nfound += 1;
    dfound += (unsigned long long)deg;
  }
  wave_stage(G, S, qn, win, v, deg);
}

// Top-down level.  Workgroups take one of three roles by id:
//   [0, nb_small)                 thread per vertex of degree <= t1; the
//                                 lanes of a wavefront step through their
//                                 rows in lock-step;
//   [nb_small, nb_small+nb_med)   wavefront per vertex of degree in (t1, t2],
//                                 reading the row 64 neighbours at a time;
//   the rest                      workgroup per t2-edge chunk of a larger
//                                 vertex.

template <class RowT>
__device__ __forceinline__ TdLevel td_level_state(const DevG<RowT> &G, const Ctl *c) {
  TdLevel t;
  t.qcur = c->qcur;
  t.level = c->level;
  // both sets' counts are read together with the rest, then selected (no
  // load that waits for qcur)
  unsigned q[2][3];
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 3; ++b) q[s][b] = c->qcnt[s][b];
  for (int b = 0; b < 3; ++b) t.cnt[b] = t.qcur ? q[1][b] : q[0][b];
  const unsigned ch0 = c->qchunk[0], ch1 = c->qchunk[1];
  t.nchunk = t.qcur ? ch1 : ch0;
  t.m_f = c->m_f;
  t.dist = c->dist;
  t.parent = c->parent;
  t.fbm = c->policy != BFS_POLICY_TD_ONLY ? (c->bcur ? G.bm[1] : G.bm[0]) : nullptr;
  t.fsm = (t.fbm && G.sshift >= 0 && td_keeps_summary(t.m_f, c->m_u, c->n, c->nnz)) ? (c->bcur ? G.sm[1] : G.sm[0])
                                                                                     : nullptr;
  t.sshift = G.sshift;
  t.from_bitmap = c->conv == kConvB2Q;
  return t;
}

// Expands frontier vertex u of the calling lane (`act`; h = its head record,
// row0 = its row offset) one lane per vertex: the first four neighbours are
// claimed together (their visited words, the claims and the new vertices'
// degrees are three rounds of independent requests instead of three per
// neighbour), then the rest of the row kTdUnroll neighbours at a time in
// lock-step with the wavefront.  All lanes of the wavefront call it together.
constexpr int kTdUnroll = 2;  // neighbours per lane per step in the wavefront / workgroup roles

// Claims K neighbours x[k] (-1: none) of frontier vertex u[k] per lane
// together: their visited words, the claims and the new vertices' degrees
// are three rounds of K independent requests instead of three per
// neighbour.  All lanes of the wavefront call it together.
template <int K, class RowT>
__device__ __forceinline__ void td_claim_batch(const DevG<RowT> &G, const Stage &S, const TdLevel &T, int qn,
                                               const int32_t (&x)[K], const int32_t (&u)[K],
                                               unsigned long long &nfound, unsigned long long &dfound) {
  bool win[K];
  if (G.td_visited == BFS_TD_VISITED_BITMAP) {
    // (32-bit halves of the visited words: half the registers of 64-bit ones)
    uint32_t *vis32 = reinterpret_cast<uint32_t *>(G.vis);
    uint32_t w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] = x[k] < 0 ? ~0u : (T.m_f < kPreloadMinEdges ? 0u : vis32[x[k] >> 5]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t bit = x[k] >= 0 ? 1u << (x[k] & 31) : 0u;
      win[k] = false;
      if (x[k] >= 0 && !(w[k] & bit)) win[k] = !(atomicOr(vis32 + (x[k] >> 5), bit) & bit);
    }
  } else if (G.td_visited == BFS_TD_DIST_CAS) {  // Section 2, BFS-Conventional
#pragma unroll
    for (int k = 0; k < K; ++k) win[k] = x[k] >= 0 && atomicCAS(T.dist + x[k], -1, T.level + 1) == -1;
  } else {  // Section 2, BFS-NonAtomic (either form): a plain test, duplicates allowed
    int32_t d[K];
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = x[k] >= 0 ? dist_test_load(G, T.dist + x[k]) : 0;
#pragma unroll
    for (int k = 0; k < K; ++k) win[k] = x[k] >= 0 && d[k] < 0;
  }
  int32_t dv[K];  // the new vertices' degrees (their queue class and the next m_f)
#pragma unroll
  for (int k = 0; k < K; ++k) dv[k] = win[k] && !G.classless ? G.head[x[k]].x : 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (win[k]) {
      // streaming stores, plain: every writer of x[k] stores this same value
      dist_store(G, T.dist + x[k], T.level + 1);
      if (T.parent) __builtin_nontemporal_store(u[k], gptr(T.parent + x[k]));
      fbm_set(T.fbm, T.fsm, T.sshift, x[k]);
      nfound += 1;
      dfound += (unsigned long long)dv[k];
    }
    wave_stage(G, S, qn, win[k], x[k], (int64_t)dv[k]);
  }
}

template <class RowT>
__device__ __forceinline__ void td_expand_lane(const DevG<RowT> &G, const Stage &S, const TdLevel &T, int qn,
                                               bool act, int32_t u, const int4 &h, int64_t row0,
                                               unsigned long long &nfound, unsigned long long &dfound) {
  const int64_t deg = act ? h.x : 0;
  {
    // the three head neighbours and the row's fourth entry (read from the
    // row while the head record is in hand) are claimed together, so rows of
    // up to four take one round of claims (a lattice's rows)
    const int32_t x[4] = {act ? h.y : -1, act ? h.z : -1, act ? h.w : -1, deg > 3 ? G.col[row0 + 3] : -1};
    const int32_t uu[4] = {u, u, u, u};
    td_claim_batch<4>(G, S, T, qn, x, uu, nfound, dfound);
  }
  for (int64_t j = 4; __ballot(j < deg); j += kTdUnroll) {  // rest of the row; j is wave-uniform
    int32_t x[kTdUnroll], uu[kTdUnroll];
#pragma unroll
    for (int q = 0; q < kTdUnroll; ++q) {
      x[q] = j + q < deg ? G.col[row0 + j + q] : -1;
      uu[q] = u;
    }
    td_claim_batch<kTdUnroll>(G, S, T, qn, x, uu, nfound, dfound);
  }
}


// Wavefronts per medium vertex: as many as the role has per queued vertex,
// at most one per kWave * kTdUnroll edges of the longest row it can hold:
// a medium row (t2 edges at most) and no longer than the whole frontier's
// degree sum m_f (so a small level keeps a single workgroup and its
// single-workgroup decide).
__host__ __device__ inline int64_t medium_split(int64_t cnt, int64_t waves, int64_t t2, int64_t m_f) {
  if (cnt <= 0) return 1;
  constexpr int64_t step = kWave * kTdUnroll;
  const int64_t rows = m_f < t2 ? m_f : t2;
  const int64_t most = (rows + step - 1) / step;
  const int64_t k = waves / cnt;
  const int64_t kpv = k < most ? k : most;
  return kpv < 1 ? 1 : kpv;
}

// One top-down level for workgroup `blk` of `nblk`.  Roles by workgroup:
//   [0, nb_small)                 thread per vertex of degree <= t1;
//   [nb_small, nb_small+nb_med)   wavefront per vertex of degree in (t1, t2],
//                                 reading the row 64 neighbours at a time;
//   the rest                      workgroup per t2-edge chunk of a larger
//                                 vertex.
// Ends with the staged queue entries flushed and the workgroup's counts in
// `counts`.  All threads of the workgroup call it.
template <class RowT>
__device__ __forceinline__ void td_level(const DevG<RowT> &G, const TdLevel &T, const Stage &S, int blk,
                                         int nblk, int nb_small, int nb_med,
                                         unsigned long long (&counts)[2]) {
  const int qc = T.qcur, qn = qc ^ 1;
  const int lane = lane_id();
  const int wib = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  unsigned long long nfound = 0, dfound = 0;
  // Every role iterates in workgroup-uniform rounds so that the staging
  // buffers can be flushed between rounds.
  if (blk < nb_small) {
    const int64_t cnt = T.cnt[kSmall];
    const int32_t *q = qc ? G.qs[1] : G.qs[0];
    const int64_t step = (int64_t)nb_small * blockDim.x;
    for (int64_t round = (int64_t)blk * blockDim.x; round < cnt; round += step) {
      const int64_t i = round + wib * kWave + lane;
      bool act = i < cnt;
      const int32_t u = act ? ld_x(q + i, G.pers) : 0;
      if (act && G.slot) act = ld_x(G.slot + u, G.pers) == (int32_t)i;  // culled duplicate: expand only the recorded copy
      if (G.nb4) {  // rows of at most four: the whole row in one record
        int4 r4 = make_int4(-1, -1, -1, -1);
        if (act) {
          r4 = G.nb4[u];
          if (G.classless)  // this level's m_f
            dfound += (unsigned long long)((r4.x >= 0) + (r4.y >= 0) + (r4.z >= 0) + (r4.w >= 0));
          fbm_clear(T.fbm, u);
        }
        const int32_t x[4] = {r4.x, r4.y, r4.z, r4.w};
        const int32_t uu[4] = {u, u, u, u};
        td_claim_batch<4>(G, S, T, qn, x, uu, nfound, dfound);
      } else {
        int4 h = make_int4(0, -1, -1, -1);
        int64_t row0 = 0;
        if (act) {
          h = G.head[u];  // degree and first three neighbours
          if (G.classless) dfound += (unsigned long long)h.x;  // this level's m_f
          row0 = (int64_t)G.rp[u];  // issued together with the head load
          fbm_clear(T.fbm, u);
        }
        td_expand_lane(G, S, T, qn, act, u, h, row0, nfound, dfound);
      }
      stage_flush(G, S, qn, true);
    }
  } else if (blk < nb_small + nb_med) {
    const int64_t cnt = T.cnt[kMedium];
    const int32_t *q = qc ? G.qm[1] : G.qm[0];
    const int64_t waves = (int64_t)nb_med * wpb;
    // kpv wavefronts share each row (interleaved steps) when the queue is
    // shorter than the role's wavefronts
    const int64_t kpv = medium_split(cnt, waves, G.t2, T.m_f);
    const int64_t items = cnt * kpv;
    for (int64_t round = (int64_t)(blk - nb_small) * wpb; round < items; round += waves) {
      const int64_t it = round + wib;
      const int64_t i = it / kpv, sub = it - i * kpv;
      const int32_t u = it < items ? ld_x(q + i, G.pers) : -1;  // uniform within the wavefront
      if (u >= 0 && (!G.slot || ld_x(G.slot + u, G.pers) == (int32_t)i)) {  // (culled duplicates skip)
        if (lane == 0 && sub == 0) fbm_clear(T.fbm, u);
        const int64_t beg = (int64_t)G.rp[u], end = (int64_t)G.rp[u + 1];
        for (int64_t b = beg + sub * kWave * kTdUnroll; b < end; b += (int64_t)kWave * kTdUnroll * kpv) {
          int32_t x[kTdUnroll], uu[kTdUnroll];
#pragma unroll
          for (int q = 0; q < kTdUnroll; ++q) {
            const int64_t j = b + q * kWave + lane;
            x[q] = j < end ? G.col[j] : -1;
            uu[q] = u;
          }
          td_claim_batch<kTdUnroll>(G, S, T, qn, x, uu, nfound, dfound);
        }
      }
      stage_flush(G, S, qn, true);
    }
  } else {
    // Large vertices: the queue holds one entry per vertex, {chunk count,
    // vertex}; this role's workgroups take the chunks round-robin by index
    // over the entries in queue order.  Every workgroup reads the entries a
    // window at a time, with the prefix sums of their chunk counts, and
    // finds the vertex of each of its chunks there.
    const int64_t nlv = T.cnt[kLarge];
    const uint64_t *q = qc ? G.ql[1] : G.ql[0];
    const int64_t nbl = (int64_t)nblk - nb_small - nb_med;
    const int64_t r = blk - nb_small - nb_med;
    __shared__ unsigned wtot;
    int64_t cbase = 0;  // chunk index of the window's first chunk
    // (the first chunk of this workgroup at or after cbase is
    // cbase + (r - cbase) mod nbl; past the total, the workgroup is done)
    for (int64_t w0 = 0; w0 < nlv && cbase + ((r - cbase % nbl) + nbl) % nbl < T.nchunk;
         w0 += blockDim.x) {  // workgroup-uniform
      const int64_t e = w0 + threadIdx.x;
      const uint64_t ent = e < nlv ? ld_x(q + e, G.pers) : 0ull;
      const unsigned incl = block_incl_scan((unsigned)(ent >> 32));
      S.wv[threadIdx.x] = ent;
      S.wp[threadIdx.x] = incl;
      if (threadIdx.x == blockDim.x - 1) wtot = incl;
      __syncthreads();
      const int64_t tot = wtot;
      const unsigned nent = (unsigned)min((int64_t)blockDim.x, nlv - w0);
      for (int64_t j = cbase + ((r - cbase % nbl) + nbl) % nbl; j < cbase + tot; j += nbl) {
        const unsigned jj = (unsigned)(j - cbase);  // (the same search in every thread)
        unsigned lo = 0, hi = nent - 1;
        while (lo < hi) {
          const unsigned mid = (lo + hi) >> 1;
          if (S.wp[mid] > jj) hi = mid;
          else lo = mid + 1;
        }
        const int32_t u = (int32_t)(uint32_t)S.wv[lo];
        const int64_t chunk = (int64_t)jj - (lo ? (int64_t)S.wp[lo - 1] : 0);
        if (chunk == 0 && threadIdx.x == 0) fbm_clear(T.fbm, u);
        const int64_t row_end = (int64_t)G.rp[u + 1];
        const int64_t beg = (int64_t)G.rp[u] + chunk * G.t2;
        const int64_t end = min(row_end, beg + (int64_t)G.t2);
        // kTdUnroll neighbours per lane per step, each step's ids coalesced;
        // the steps are workgroup-uniform, and the staging buffers are
        // emptied after a step that leaves one of them at least half full (a
        // step stages at most kTdUnroll entries per thread, so the small and
        // medium buffers never overflow; a hub's neighbours are themselves of
        // high degree, and entries past a full buffer would go to the global
        // queue with one contended atomic per wavefront)
        for (int64_t step = beg; step < end; step += (int64_t)blockDim.x * kTdUnroll) {
          const int64_t bb = step + wib * kWave * kTdUnroll;
          int32_t x[kTdUnroll], uu[kTdUnroll];
#pragma unroll
          for (int qq = 0; qq < kTdUnroll; ++qq) {
            const int64_t jn = bb + qq * kWave + lane;
            x[qq] = jn < end ? G.col[jn] : -1;
            uu[qq] = u;
          }
          td_claim_batch<kTdUnroll>(G, S, T, qn, x, uu, nfound, dfound);
          stage_flush(G, S, qn, true);
        }
      }
      cbase += tot;
      __syncthreads();  // every thread is done with the window before the next one
    }
  }
  stage_flush(G, S, qn);
  counts[0] = nfound;
  counts[1] = dfound;
}

// Top-down level whose frontier is the bitmap a bottom-up level left (the
// level after a switch back to top-down; no conversion to queues): every
// workgroup expands the frontier vertices of its own share of the words.  A
// wavefront loads 64 words with one coalesced load, compacts their set bits
// into batches of 64 in an LDS ring and loads the head records together.
// Discoveries of this level enter the same bitmap while it is read, so a set
// bit is a frontier vertex only if its distance is this level's (written by
// an earlier level; a vertex found now holds level + 1, or -1 if that store
// is not yet visible); only those are expanded and taken out of the bitmap.
// Vertices of degree <= t1 are expanded by their lane, larger ones by the
// whole wavefront, 64 neighbours at a time.  `ring` is this wavefront's
// kCandTd-entry LDS ring.
constexpr int kCandTd = 128;

template <class RowT>
__device__ __forceinline__ void td_level_bitmap(const DevG<RowT> &G, const TdLevel &T, const Stage &S,
                                                int32_t *ring, unsigned long long (&counts)[2]) {
  const int qn = T.qcur ^ 1;
  const int lane = lane_id();
  unsigned long long nfound = 0, dfound = 0;
  uint64_t *fbm = T.fbm;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * wpb;
  const int64_t gw = xcd_block(gridDim.x) * wpb + (threadIdx.x >> 6);
  const int64_t per = (G.words + nw - 1) / nw;
  const int64_t w0 = gw * per;
  const int64_t w1 = min(G.words, w0 + per);
  // expands the `cnt` ring entries from `head`
  auto batch = [&](unsigned head, int cnt) {
    bool act = lane < cnt;
    int32_t u = 0;
    int4 h = make_int4(0, -1, -1, -1);
    int64_t row0 = 0;
    int32_t du = -1;
    if (act) {
      u = ring[(head + lane) & (kCandTd - 1)];
      du = *gptr(T.dist + u);
      h = G.head[u];
      row0 = (int64_t)G.rp[u];
    }
    act = act && du == T.level;  // a frontier vertex, not one found this level
    if (act) fbm_clear(fbm, u);
    const bool big = act && h.x > G.t1;
    td_expand_lane(G, S, T, qn, act && !big, u, h, row0, nfound, dfound);
    uint64_t bm = __ballot(big);
    while (bm) {  // larger rows: the whole wavefront, 64 neighbours at a time
      const int l = __ffsll((unsigned long long)bm) - 1;
      bm &= bm - 1;
      const int32_t ub = __shfl(u, l);
      const int64_t beg = __shfl(row0, l);
      const int64_t end = beg + __shfl(h.x, l);
      for (int64_t b = beg; b < end; b += kWave) {
        const int64_t j = b + lane;
        const bool has = j < end;
        const int32_t v = has ? G.col[j] : 0;
        td_visit(G, S, qn, T, has, ub, v, T.m_f >= kPreloadMinEdges, nfound, dfound);
      }
    }
  };
  for (int64_t r = 0; r < per; r += kWave) {  // workgroup-uniform rounds of 64 words
    const int64_t sr = w0 + r;
    const uint64_t wd = sr + lane < w1 ? fbm[sr + lane] : 0ull;
    uint64_t nz = __ballot(wd != 0ull);
    unsigned ch = 0, ct = 0;  // ring head / tail (wave-uniform)
    while (nz) {
      const int k = __builtin_ctzll(nz);
      nz &= nz - 1;
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)wd, k);
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(wd >> 32), k);
      const uint64_t bits = ((uint64_t)hi << 32) | lo;
      if ((bits >> lane) & 1ull) ring[(ct + lanes_below(bits)) & (kCandTd - 1)] = (int32_t)((sr + k) * kWave + lane);
      ct += (unsigned)__popcll(bits);
      if (ct - ch >= (unsigned)kWave) {
        batch(ch, kWave);
        ch += kWave;
      }
    }
    if (ct != ch) batch(ch, (int)(ct - ch));
    stage_flush(G, S, qn, true);
  }
  stage_flush(G, S, qn);
  counts[0] = nfound;
  counts[1] = dfound;
}

// Launch options of the level kernel.
enum LevelMode : int32_t {
  kFusedDecide = 1  // the last workgroup applies the decide step
};

// End of a direction kernel: the workgroup's K counts reach the decide
// step, either as this workgroup's slot of the partials array (a later
// kernel reduces them) or, with kFusedDecide, through the fused decide step,
// which needs no memory fence (a release fence at device scope writes back
// the XCD's whole L2, far too costly once per workgroup):
//   1. thread 0 adds the workgroup's counts to the accumulators of its group
//      (blockIdx.x modulo kArriveGroups: consecutive workgroups go to
//      different XCDs, so no accumulator takes more than a 1/kArriveGroups
//      share) with device-scope atomics and waits for them to complete;
//   2. it then arrives on its group's counter; the last arrival of a group
//      arrives on the counter over the groups;
//   3. the last arrival of all collects the totals by exchanging the
//      accumulators with zero (completed atomics, so every count is there),
//      resets the counters, and applies the decide step.
// A level run by a single workgroup reduces in LDS and decides at once.
// (Small grids once released per-workgroup slots with a fence instead; the
// atomics are faster for them too: 12 % less per level on the lattice.)
// All threads of the workgroup call it.

// `rank` numbers the nactive workgroups that take part (workgroups with no
// work in the level exit before and do not arrive); `level` is the level
// being run, or -1 (then the deciding thread reads it).
template <int K, class RowT>
__device__ __forceinline__ void end_level(const DevG<RowT> &G, int32_t mode, const unsigned long long (&v)[K],
                                          unsigned rank, unsigned nactive, int32_t level) {
  if (!(mode & kFusedDecide)) {
    block_partials<K>(G, v, rank);
    return;
  }
  uint32_t *arrive = reinterpret_cast<uint32_t *>(G.partials + kArriveOffset);
  constexpr int kLineU32 = 2 * kLineU64;
  if (nactive == 1) {  // the only workgroup of the level: reduce in LDS and decide
    __shared__ unsigned long long one[K][16];
    const int w = threadIdx.x >> 6;
    if (threadIdx.x == 0) {  // first (see decide_apply), overlapping the reduction
      if (level < 0) level = G.ctl->level;
      (void)__hip_atomic_exchange(&G.ctl->level, level + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const unsigned long long sum = wave_sum(v[k]);
      if (lane_id() == 0) one[k][w] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot[kPartials] = {0, 0, 0, 0};
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot[k] += one[k][i];
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      decide_apply(G.ctl, G.recs, tot, level);
    }
    return;
  }
  __shared__ unsigned long long part[K][16];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const unsigned long long sum = wave_sum(v[k]);
    if (lane_id() == 0) part[k][w] = sum;
  }
  __syncthreads();
  if (threadIdx.x >= kWave) return;  // wave 0 finishes; its lanes work in parallel
  const int lane = threadIdx.x;
  unsigned long long *acc = G.partials + kAccOffset;
  const unsigned grp = rank % kArriveGroups;
  const unsigned gsize = (nactive - grp + kArriveGroups - 1) / kArriveGroups;
  const unsigned ngroups = nactive < (unsigned)kArriveGroups ? nactive : (unsigned)kArriveGroups;
  if (lane < K) {
    unsigned long long t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[lane][i];
    if (t) atomicAdd(&acc[(grp * kPartials + lane) * kLineU64], t);
  }
  // the adds must have completed before this workgroup is counted
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  unsigned arrived = 0;
  if (gsize > 1) {  // (a group of one workgroup goes straight to the top counter)
    if (lane == 0) arrived = atomicAdd(&arrive[grp * kLineU32], 1u);
    if (__shfl(arrived, 0) != gsize - 1) return;
    if (lane == 0) atomicExch(&arrive[grp * kLineU32], 0u);
  }
  if (lane == 0) arrived = atomicAdd(&arrive[kArriveGroups * kLineU32], 1u);
  if (__shfl(arrived, 0) != ngroups - 1) return;
  if (lane == 0) {
    if (level < 0) level = G.ctl->level;
    // first (see publish_level); the wait below covers it
    (void)__hip_atomic_exchange(&G.ctl->level, level + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicExch(&arrive[kArriveGroups * kLineU32], 0u);
  }
  // lane g * kPartials + k takes accumulator k of group g; sums over the
  // lanes of equal k (lane mod kPartials) give the totals
  static_assert((kPartials & (kPartials - 1)) == 0 && kArriveGroups * kPartials <= kWave,
                "the lane mapping needs a power-of-two kPartials and one lane per accumulator");
  unsigned long long x = 0;
  if ((unsigned)lane < ngroups * kPartials) x = atomicExch(&acc[(size_t)lane * kLineU64], 0ull);
#pragma unroll
  for (int o = kPartials; o < kWave; o <<= 1) x += __shfl_xor(x, o);
  unsigned long long tot[kPartials];
#pragma unroll
  for (int k = 0; k < kPartials; ++k) tot[k] = __shfl(x, k);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if (lane == 0) decide_apply(G.ctl, G.recs, tot, level);
}

// Persistent top-down search (top-down-only policies): every level of the
// search in one cooperative launch, with no cache write-back or invalidation
// between levels.  Data one level hands to the next crosses XCDs through
// the device-coherent level of the memory system: queue entries (and culled
// copies' slots and plainly tested distances) are written and read with
// agent-scope accesses (G.pers), counts are added with atomics, and the
// control block is read and written with agent-scope accesses.  The
// distances and parents of the bitmap and compare-and-swap visited tests
// are not read during the search.  A level ends like this:
//   1. every thread waits for its own stores to complete; the workgroup adds
//      its degree sum to an accumulator, waits for that, then adds
//      (found << 11) + 1 to the arrival word with one returning atomic;
//   2. the workgroup whose arrival completes the count (the word's low bits
//      reach the grid size) takes the totals, clears both words, applies the
//      decide step with agent-scope accesses, waits for them, and bumps the
//      generation number; the others poll it (bounded: a wait that outlasts
//      kPersistSpinLimit polls ends the search with an error flag).
constexpr uint64_t kPersistSpinLimit = 1ull << 26;
constexpr int kArrivalBits = 11;  // arrivals per level < 2^11 (at most kMaxBlocks workgroups)

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ldc(const T &f) {
  return __hip_atomic_load(const_cast<T *>(&f), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void stc(T &f, T v) {
  __hip_atomic_store(&f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The decide step of a top-down-only level inside the persistent kernel
// (decide_apply's top-down branch, with device-coherent control-block
// accesses).  Every field is loaded in one batch of independent loads and
// every store issued in one batch, so the step costs two round trips to the
// coherence point rather than one per field.  One thread.
__device__ void decide_persistent(Ctl *c, LevelRec *recs, int64_t found, int64_t fdeg, unsigned qcap0,
                                  unsigned qcap1, bool classless) {
  const int32_t L = ldc(c->level);
  const int32_t qcur = ldc(c->qcur);
  const int32_t rec_cap = ldc(c->rec_cap);
  const int32_t over = ldc(c->overflow);
  const int64_t n_f = ldc(c->n_f), m_f = ldc(c->m_f), m_u = ldc(c->m_u);
  const int64_t sum_mf = ldc(c->sum_mf), reached = ldc(c->reached);
  unsigned q[2][3];
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 3; ++b) q[s][b] = ldc(c->qcnt[s][b]);
  // (classless: fdeg is this level's own m_f, summed while expanding it)
  const int64_t mf = classless ? fdeg : m_f;
  const int64_t mu = classless ? m_u - fdeg : m_u;
  const int32_t nq = qcur ^ 1;  // the next frontier's queue set
  const unsigned *qn = nq ? q[1] : q[0];
  const bool overflow = over || qn[kSmall] > qcap0 || qn[kMedium] > qcap0 || qn[kLarge] > qcap1;
  const bool end = overflow || found == 0;
  if (L < rec_cap) {  // (read by the host after the kernel)
    LevelRec r;
    r.level = L;
    r.dir = kTD;
    r.n_f = n_f;
    r.m_f = mf;
    r.m_u = mu;
    r.found = found;
    r.scanned = 0;
    r.examined = 0;
    recs[L] = r;
  }
  stc(c->levels_done, L + 1);
  stc(c->sum_mf, sum_mf + mf);
  stc(c->reached, reached + found);
  for (int b = 0; b < 3; ++b) stc(c->qcnt[qcur][b], 0u);  // emptied for the level after
  stc(c->qchunk[qcur], 0u);
  stc(c->qcur, nq);
  if (overflow) stc(c->overflow, 1);
  if (end) {
    stc(c->conv, (int32_t)kConvNone);
    stc(c->done, 1);
  } else {
    stc(c->n_f, found);
    stc(c->m_f, classless ? (int64_t)0 : fdeg);
    stc(c->m_u, classless ? mu : m_u - fdeg);
  }
  stc(c->level, L + 1);
}

template <class RowT>
__global__ void __launch_bounds__(1024) k_td_persistent(DevG<RowT> G, int32_t nb_small, int32_t nb_med) {
  extern __shared__ __align__(16) char lds[];
  __shared__ unsigned long long wsum[2][16];
  __shared__ int go;
  Ctl *c = G.ctl;
  unsigned long long *acc = G.partials + kAccOffset;             // degree sum of the level
  unsigned long long *arrive = G.partials + kArriveOffset;       // (found << 11) + arrivals
  uint32_t *gen = reinterpret_cast<uint32_t *>(G.partials + kArriveOffset + kLineU64);  // levels released
  for (int64_t it = 0; it <= G.n; ++it) {
    // The level's state in one round of loads (read after the release every
    // workgroup saw): both queue sets' counts are read and the current one
    // selected, so no load waits for another.
    const int32_t done = ldc(c->done);
    TdLevel T;
    T.qcur = ldc(c->qcur);
    T.level = ldc(c->level);
    T.m_f = ldc(c->m_f);
    unsigned q[2][3], qch[2];
    for (int s2 = 0; s2 < 2; ++s2) {
      for (int b = 0; b < 3; ++b) q[s2][b] = ld_agent(&c->qcnt[s2][b]);
      qch[s2] = ld_agent(&c->qchunk[s2]);
    }
    if (done) break;  // uniform
    for (int b = 0; b < 3; ++b) T.cnt[b] = T.qcur ? q[1][b] : q[0][b];
    T.nchunk = T.qcur ? qch[1] : qch[0];
    T.dist = c->dist;  // constant for the whole search
    T.parent = c->parent;
    T.fbm = nullptr;  // top-down only: no frontier bitmap to keep
    T.fsm = nullptr;
    T.sshift = G.sshift;
    T.from_bitmap = false;
    const Stage S = stage_open(lds);
    unsigned long long counts[2];
    td_level(G, T, S, blockIdx.x, gridDim.x, nb_small, nb_med, counts);
    // this workgroup's stores are complete before it arrives
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const int w = threadIdx.x >> 6;
    const unsigned long long f = wave_sum(counts[0]), d = wave_sum(counts[1]);
    if (lane_id() == 0) {
      wsum[0][w] = f;
      wsum[1][w] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tf = 0, td = 0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        tf += wsum[0][i];
        td += wsum[1][i];
      }
      if (td) atomicAdd(acc, td);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      const unsigned long long mine = (tf << kArrivalBits) + 1ull;
      const unsigned long long old = atomicAdd(arrive, mine);
      const unsigned long long now = old + mine;
      int ended = 0;
      if ((now & ((1ull << kArrivalBits) - 1)) == gridDim.x) {  // the last arrival: decide
        const int64_t found = (int64_t)(now >> kArrivalBits);
        const int64_t fdeg = (int64_t)atomicExch(acc, 0ull);
        atomicExch(arrive, 0ull);
        decide_persistent(c, G.recs, found, fdeg, G.qcap, G.lcap, G.classless != 0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint32_t g0 = (uint32_t)it;  // releases so far
        uint64_t spins = 0;
        while (ld_agent(gen) == g0) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kPersistSpinLimit) {  // a workgroup that never arrives: stop everyone
            stc(c->overflow, 2);
            stc(c->done, 1);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ended = 1;
            break;
          }
        }
      }
      go = !ended;
    }
    __syncthreads();
    if (!go) break;
  }
  // the last decide publishes the final state for the host (one thread of
  // the deciding workgroup, after invalidating its XCD's view)
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    // workgroup 0 waits until every level has been released (it left the
    // loop after seeing done), then publishes
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    publish(c);
  }
}

// Bottom-up level (Section 2, Listing 2: every unvisited vertex looks for a
// frontier neighbour and stops at the first).  A wavefront owns a contiguous
// run of 64-bit visited words (64 vertices each), taken 64 words at a time:
//   1. the 64 visited words are loaded with one coalesced load (a lane each);
//      words with no unvisited vertex are skipped without any other work;
//   2. the unvisited vertices of the remaining words are compacted, in word
//      order, into a per-wavefront candidate ring in LDS, so every lane of a
//      batch holds a real candidate whatever the density of unvisited
//      vertices (dense early levels and sparse late ones cost the same per
//      candidate);
//   3. each batch of up to 128 candidates (two per lane) loads its head
//      records (degree and first three neighbours) and tests them against
//      the frontier bitmap (the second and third only where the first
//      misses); the next batch's head records are already in flight while a
//      batch is resolved;
//   4. candidates that miss and have longer rows go to a deferred ring; once
//      64 have gathered, the wavefront scans the rest of those rows laid end
//      to end, a lane per neighbour, two 64-neighbour steps in flight; rows
//      longer than tbu by the whole wavefront with a ballot early exit;
//   5. the found masks collect in LDS and are written as next-frontier and
//      visited words with one coalesced store per run.
// `examined` counts neighbours up to and including the first hit.
// A bottom-up wavefront resolves its candidates kBuSub * 64 at a time (lane
// l holds candidates l, l + 64, ...), so the frontier-word gathers of kBuSub
// batches are in flight together.
constexpr int kBuSub = 2;
constexpr int kBuBatch = kBuSub * kWave;
constexpr int kCand = 256;  // candidate ring: < kBuBatch waiting + 64 from one word
constexpr int kDefer = 128;  // deferred ring: < 64 waiting + 64 from one sub-batch

struct BuWaveLds {
  int32_t cand[kCand];
  int32_t crank[kCand];  // the candidate's index in the compacted head records
  uint64_t live[kWave];  // the run's non-isolated masks
  uint32_t rank[kWave];  // and compacted-record offsets, one per word
  int32_t dv[kDefer];
  int32_t ddeg[kDefer];
  int32_t dcr[kDefer];   // the deferred vertex's index in the compacted records
  uint64_t mask[kWave];
};

__host__ __device__ constexpr size_t bu_lds_bytes(int bs) { return (size_t)(bs / kWave) * sizeof(BuWaveLds); }


// The frontier bitmap a bottom-up level tests, and optionally an LDS copy
// of its occupancy summary: a neighbour whose word's summary bit is clear is
// not in the frontier, and is rejected without the random read of its
// frontier word (with a small frontier, most of the level's reads).
struct Front {
  const uint32_t *bits;  // the frontier bitmap as 32-bit words
  const uint64_t *lsum;  // the summary in LDS, or null (test every neighbour's word)
  int32_t sshift;
};

__device__ __forceinline__ bool may_be_front(const Front &F, int32_t x) {
  if (!F.lsum) return true;
  const uint32_t sb = ((uint32_t)x >> 6) >> F.sshift;
  return (F.lsum[sb >> 6] >> (sb & 63)) & 1ull;
}

// The frontier word holding vertex x (x >= 0), or 0 where the summary rules
// it out.
__device__ __forceinline__ uint32_t front_word(const Front &F, int32_t x) {
  return may_be_front(F, x) ? F.bits[x >> 5] : 0u;
}

__device__ __forceinline__ bool front_bit(const Front &F, int32_t x) {
  return (front_word(F, x) >> (x & 31)) & 1u;
}

// Per-lane counters of a bottom-up level (a lane handles far fewer than
// 2^32 candidates; degree sums need 64 bits).
struct BuCount {
  uint32_t found = 0, scan = 0;
  unsigned long long fdeg = 0, exam = 0;
};

// Records a bottom-up find: v's distance and parent (streaming stores: the
// level does not read them again, and left in the caches they would take
// room from the frontier words and head records), its counts, and its bit
// in the run's found masks.
template <class RowT>
__device__ __forceinline__ void bu_found(BuWaveLds &W, int32_t v, int32_t deg, int32_t hit, int64_t sr,
                                         int32_t level, int32_t *dist, int32_t *parent, BuCount &C) {
  __builtin_nontemporal_store(level + 1, gptr(dist + v));
  if (parent) __builtin_nontemporal_store(hit, gptr(parent + v));
  C.found += 1;
  C.fdeg += (unsigned long long)deg;
  atomicOr(reinterpret_cast<unsigned long long *>(&W.mask[(v >> 6) - sr]), 1ull << (v & 63));
}

// Scans the rows of the `cnt` (<= 64) deferred vertices from ring slot
// `head` past their head records.  The rows' remaining neighbours are laid
// end to end and read 64 at a time, a lane per neighbour, so a step reads
// whole stretches of rows whatever their lengths (one row per lane would take
// as many steps as the longest row needs while the other lanes idle).  The
// neighbour ids of kDrainSteps such steps are loaded before any of them is
// tested, so a wavefront has that many steps' loads in flight instead of
// one.  Each row takes its first frontier neighbour in row order (steps in
// order, then lanes); lanes of a row that had already hit when the steps
// were loaded read nothing more.  Records the finds.
constexpr int kDrainSteps = 2;

template <class RowT>
__device__ __forceinline__ void bu_drain(const DevG<RowT> &G, BuWaveLds &W, unsigned head, unsigned cnt,
                                         const Front &front, int64_t sr, int32_t level, int32_t *dist,
                                         int32_t *parent, BuCount &C) {
  const int lane = lane_id();
  const bool act = (unsigned)lane < cnt;
  const unsigned slot = (head + lane) & (kDefer - 1);
  int32_t v = 0, deg = 0;
  int64_t from = 0;  // the row's first neighbour past the head record
  if (act) {
    v = W.dv[slot];
    deg = W.ddeg[slot];
    from = (G.rpc ? (int64_t)G.rpc[W.dcr[slot]] : (int64_t)G.rp[v]) + 3;
  }
  const int32_t len = act ? deg - 3 : 0;  // >= 1: deferred rows are longer than the head
  int32_t incl = len;  // inclusive prefix sum of the lengths over the lanes
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const int32_t off = incl - len;  // the row's first position in the packed sequence
  const int32_t total = __shfl(incl, kWave - 1);
  bool found = false;
  int32_t hit = -1, ex = deg;
  const uint64_t upto = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;  // lanes <= this one
  for (int32_t p0 = 0; p0 < total; p0 += kWave * kDrainSteps) {  // uniform
    int32_t x[kDrainSteps];
    bool h[kDrainSteps];
    const bool done0 = found;  // rows that hit in an earlier round read nothing more
#pragma unroll
    for (int u = 0; u < kDrainSteps; ++u) {
      // position p + lane belongs to the last row that starts at or before it
      const int32_t p = p0 + u * kWave;
      const bool starts = act && off >= p && off < p + kWave;
      const uint64_t sbits = wave_or(starts ? 1ull << (off - p) : 0ull);
      const int r = __popcll(__ballot(act && off < p)) + __popcll(sbits & upto) - 1;
      const int32_t e = p + lane;
      const int64_t rfrom = __shfl(from, r);
      const int32_t roff = __shfl(off, r);
      const bool rdone = __shfl((int)done0, r) != 0;
      x[u] = -1;
      if (e < total && !rdone) x[u] = G.col[rfrom + (e - roff)];
    }
#pragma unroll
    for (int u = 0; u < kDrainSteps; ++u) h[u] = x[u] >= 0 && front_bit(front, x[u]);
#pragma unroll
    for (int u = 0; u < kDrainSteps; ++u) {
      const int32_t p = p0 + u * kWave;
      const uint64_t hm = __ballot(h[u]);
      // each unfinished row takes the first hit within its own lanes
      int f = -1;
      if (act && !found) {
        const int32_t lo = max(off, p) - p, hi = min(off + len, p + kWave) - p;  // its lanes [lo, hi)
        if (lo < hi) {
          const uint64_t seg = (hi == kWave ? ~0ull : (1ull << hi) - 1) & ~((1ull << lo) - 1);
          const uint64_t mh = hm & seg;
          if (mh) f = __builtin_ctzll(mh);
        }
      }
      const int32_t xf = __shfl(x[u], f < 0 ? 0 : f);
      if (f >= 0) {
        found = true;
        hit = xf;
        ex = 3 + (p + f - off) + 1;
      }
    }
  }
  if (act) C.exam += (unsigned long long)ex;
  if (found) bu_found<RowT>(W, v, deg, hit, sr, level, dist, parent, C);
}

// Scans the rows of the lanes in `lanes` (vertices longer than tbu) one
// after the other, each by the whole wavefront 64 neighbours at a time past
// its head record, stopping at the row's first frontier neighbour.  Records
// the finds.
template <class RowT>
__device__ __forceinline__ void bu_long_rows(const DevG<RowT> &G, BuWaveLds &W, uint64_t lanes, int32_t v,
                                             int32_t deg, const Front &front, int64_t sr, int32_t level,
                                             int32_t *dist, int32_t *parent, BuCount &C) {
  const int lane = lane_id();
  const bool mine = (lanes >> lane) & 1ull;
  int64_t row0 = 0;
  if (mine) row0 = (int64_t)G.rp[v];
  bool found = false;
  int32_t hit = -1;
  int64_t ex = deg;
  while (lanes) {
    const int l = __ffsll((unsigned long long)lanes) - 1;
    lanes &= lanes - 1;
    const int64_t r0 = __shfl(row0, l);
    const int64_t e0 = r0 + __shfl(deg, l);
    int64_t exl = e0 - r0;
    int32_t hitl = -1;
    // kDrainSteps steps of 64 neighbours loaded, then tested in order
    for (int64_t b0 = r0 + 3; b0 < e0 && hitl < 0; b0 += (int64_t)kWave * kDrainSteps) {  // uniform
      int32_t x[kDrainSteps];
#pragma unroll
      for (int u = 0; u < kDrainSteps; ++u) {
        const int64_t j = b0 + u * kWave + lane;
        x[u] = j < e0 ? G.col[j] : -1;
      }
      bool h[kDrainSteps];
#pragma unroll
      for (int u = 0; u < kDrainSteps; ++u) h[u] = x[u] >= 0 && front_bit(front, x[u]);
#pragma unroll
      for (int u = 0; u < kDrainSteps; ++u) {
        const uint64_t hb = __ballot(h[u]);
        if (hb && hitl < 0) {  // uniform
          const int f = __ffsll((unsigned long long)hb) - 1;
          hitl = __shfl(x[u], f);
          exl = b0 + u * kWave - r0 + f + 1;
        }
      }
    }
    if (lane == l) {
      ex = exl;
      if (hitl >= 0) {
        found = true;
        hit = hitl;
      }
    }
  }
  if (mine) C.exam += (unsigned long long)ex;
  if (found) bu_found<RowT>(W, v, deg, hit, sr, level, dist, parent, C);
}

// Resolves one batch of `cnt` (<= kBuBatch) candidates (candidate
// k * 64 + lane is vertex v[k] with head record h[k] in lane `lane`): tests
// the head neighbours of all of them together, then, sub-batch by sub-batch,
// records the finds, scans rows longer than tbu at once and defers the rest
// of the longer rows (draining 64 deferred rows when that many wait, and
// every deferred row after the `last` batch of a run).
template <class RowT>
__device__ __forceinline__ void bu_resolve(const DevG<RowT> &G, BuWaveLds &W, const int32_t (&v)[kBuSub],
                                           const int32_t (&cr)[kBuSub], const int4 (&h)[kBuSub], int cnt,
                                           const Front &front, int64_t sr, int32_t level, int32_t *dist,
                                           int32_t *parent, unsigned &dh, unsigned &dc, bool last, BuCount &C) {
  const int lane = lane_id();
  bool act[kBuSub];
#pragma unroll
  for (int k = 0; k < kBuSub; ++k) act[k] = lane + k * kWave < cnt;
  // the second and third head neighbours are tested only where the first
  // misses (with hub-first rows most finds are at the first, and the
  // frontier-bit gathers are the level's largest request count)
  uint32_t f0[kBuSub], f1[kBuSub], f2[kBuSub];
#pragma unroll
  for (int k = 0; k < kBuSub; ++k) {
    f0[k] = f1[k] = f2[k] = 0;
    if (act[k]) f0[k] = front_word(front, h[k].y);  // degree >= 1: the first neighbour exists
  }
#pragma unroll
  for (int k = 0; k < kBuSub; ++k) {
    if (act[k] && !((f0[k] >> (h[k].y & 31)) & 1u)) {
      if (h[k].z >= 0) f1[k] = front_word(front, h[k].z);
      if (h[k].w >= 0) f2[k] = front_word(front, h[k].w);
    }
  }
#pragma unroll
  for (int k = 0; k < kBuSub; ++k) {
    bool found = false, defer = false, longrow = false;
    int32_t hit = -1;
    const int4 hk = h[k];
    if (act[k]) {
      int32_t ex = hk.x;
      if ((f0[k] >> (hk.y & 31)) & 1u) {
        found = true; hit = hk.y; ex = 1;
      } else if (hk.z >= 0 && ((f1[k] >> (hk.z & 31)) & 1u)) {
        found = true; hit = hk.z; ex = 2;
      } else if (hk.w >= 0 && ((f2[k] >> (hk.w & 31)) & 1u)) {
        found = true; hit = hk.w; ex = 3;
      } else if (hk.x > 3) {
        (hk.x > G.tbu ? longrow : defer) = true;  // counted when its row is scanned
      }
      if (!defer && !longrow) C.exam += (unsigned long long)ex;
      C.scan += 1;
    }
    if (found) bu_found<RowT>(W, v[k], hk.x, hit, sr, level, dist, parent, C);
    const uint64_t lm = __ballot(longrow);
    if (lm) bu_long_rows(G, W, lm, v[k], hk.x, front, sr, level, dist, parent, C);
    const uint64_t dm = __ballot(defer);
    if (defer) {
      const unsigned slot = (dh + dc + lanes_below(dm)) & (kDefer - 1);
      W.dv[slot] = v[k];
      W.ddeg[slot] = hk.x;
      W.dcr[slot] = cr[k];
    }
    dc += (unsigned)__popcll(dm);
    // (fewer than 64 wait after this, so the next sub-batch fits the ring)
    while (dc >= kWave || (last && k == kBuSub - 1 && dc > 0)) {  // uniform
      const unsigned n = dc < kWave ? dc : kWave;
      bu_drain(G, W, dh, n, front, sr, level, dist, parent, C);
      dh = (dh + n) & (kDefer - 1);
      dc -= n;
    }
  }
}

template <class RowT>
__device__ __forceinline__ void bu_level(const DevG<RowT> &G, const Ctl *c, char *lds,
                                         unsigned long long (&counts)[kPartials]) {
  BuWaveLds &W = reinterpret_cast<BuWaveLds *>(lds)[threadIdx.x >> 6];
  const int bcur = c->bcur;
  uint64_t *next = bcur ? G.bm[0] : G.bm[1];
  const int32_t level = c->level;
  int32_t *dist = c->dist;
  int32_t *parent = c->parent;
  const int64_t n_f = c->n_f;
  const int lane = lane_id();
  BuCount C;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * wpb;
  const int64_t gw = xcd_block(gridDim.x) * wpb + (threadIdx.x >> 6);
  int64_t per = (G.words + nw - 1) / nw;
  // With runs of whole summary bytes (8 << sshift words, which every grid of
  // one search either has or has not), each wavefront writes the summary
  // bytes of its own run: the next frontier's summary is then exact.
  const int64_t sum_align = G.sshift >= 0 ? (int64_t)8 << G.sshift : 0;
  const bool sums = G.sshift >= 0 && per >= sum_align;
  if (sums) per = (per + sum_align - 1) / sum_align * sum_align;
  // Small frontiers leave most summary bits clear: copy the summary into LDS
  // and test it before each frontier word is read.  (Once most words hold a
  // frontier vertex the copy would save little.)
  Front front;
  front.bits = reinterpret_cast<const uint32_t *>(bcur ? G.bm[1] : G.bm[0]);
  front.lsum = nullptr;
  front.sshift = G.sshift;
  if (sums && n_f <= kSumFrontierWords * G.words && c->sum_ok[bcur]) {
    uint64_t *lsum = reinterpret_cast<uint64_t *>(lds + bu_lds_bytes(blockDim.x));
    const uint64_t *fsm = bcur ? G.sm[1] : G.sm[0];
    for (int i = threadIdx.x; i < G.swords; i += blockDim.x) lsum[i] = fsm[i];
    front.lsum = lsum;
  }
  __syncthreads();
  uint8_t *snext = sums ? reinterpret_cast<uint8_t *>(bcur ? G.sm[0] : G.sm[1]) : nullptr;
  const int64_t w_end = min(G.words, (gw + 1) * per);
  for (int64_t sr = gw * per; sr < w_end; sr += kWave) {
    const int nwd = (int)min((int64_t)kWave, w_end - sr);
    const uint64_t my_vis = lane < nwd ? G.vis[sr + lane] : ~0ull;
    W.live[lane] = lane < nwd ? ~G.iso[sr + lane] : 0ull;  // non-isolated vertices
    W.rank[lane] = lane < nwd ? G.hrank[sr + lane] : 0u;
    W.mask[lane] = 0;
    uint64_t act = __ballot(my_vis != ~0ull);  // words with an unvisited vertex
    unsigned ch = 0, ct = 0;                   // candidate ring head / tail (uniform)
    unsigned dh = 0, dc = 0;                   // deferred ring head / count
    int pc = 0;                                // candidates of the batch in flight
    int32_t pv[kBuSub], pcr[kBuSub];
    int4 ph[kBuSub];
#pragma unroll
    for (int k = 0; k < kBuSub; ++k) {
      pv[k] = 0;
      pcr[k] = 0;
      ph[k] = make_int4(0, 0, -1, -1);
    }
    for (;;) {
      if (act) {
        const int k = __builtin_ctzll(act);
        act &= act - 1;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)my_vis, k);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(my_vis >> 32), k);
        const uint64_t un = ~(((uint64_t)hi << 32) | lo);  // its unvisited vertices
        if ((un >> lane) & 1ull) {
          const unsigned slot = (ct + lanes_below(un)) & (kCand - 1);
          W.cand[slot] = (int32_t)((sr + k) * kWave + lane);
          W.crank[slot] = (int32_t)(W.rank[k] + lanes_below(W.live[k]));
        }
        ct += (unsigned)__popcll(un);
        if (ct - ch < (unsigned)kBuBatch && act) continue;  // uniform
      }
      // next batch: load its head records, then resolve the one in flight
      // (an empty next batch marks the run's last resolve)
      const int cnt = (int)min(ct - ch, (unsigned)kBuBatch);
      if (cnt == 0 && pc == 0) break;
      int32_t bv[kBuSub], bcr[kBuSub];
      int4 bh[kBuSub];
#pragma unroll
      for (int k = 0; k < kBuSub; ++k) {
        bv[k] = 0;
        bcr[k] = 0;
        bh[k] = make_int4(0, 0, -1, -1);
        if (lane + k * kWave < cnt) {
          bv[k] = W.cand[(ch + k * kWave + lane) & (kCand - 1)];
          bcr[k] = W.crank[(ch + k * kWave + lane) & (kCand - 1)];
          bh[k] = G.headc[bcr[k]];
        }
      }
      ch += cnt;
      if (pc) bu_resolve(G, W, pv, pcr, ph, pc, front, sr, level, dist, parent, dh, dc, cnt == 0, C);
#pragma unroll
      for (int k = 0; k < kBuSub; ++k) {
        pv[k] = bv[k];
        pcr[k] = bcr[k];
        ph[k] = bh[k];
      }
      pc = cnt;
    }
    // one coalesced store of the run's next-frontier and visited words
    const uint64_t m = lane < nwd ? W.mask[lane] : 0ull;
    if (lane < nwd) {
      next[sr + lane] = m;
      if (m) G.vis[sr + lane] = my_vis | m;
    }
    if (snext) {  // and the summary bytes of these words (sr is a multiple of 8 << sshift)
      const uint64_t occ = __ballot(m != 0ull);
      uint64_t sb = occ;
      if (G.sshift > 0) {
        const int g = 1 << G.sshift;
        const bool any = lane < (kWave >> G.sshift) && ((occ >> (lane * g)) & ((1ull << g) - 1)) != 0ull;
        sb = __ballot(any);
      }
      const int nbytes = (((nwd + (1 << G.sshift) - 1) >> G.sshift) + 7) >> 3;
      if (lane < nbytes) snext[((sr >> G.sshift) >> 3) + lane] = (uint8_t)(sb >> (8 * lane));
    }
  }
  counts[0] = C.found;
  counts[1] = C.fdeg;
  counts[2] = C.scan;
  counts[3] = C.exam;
}

// One level, in the direction the decide step chose: top-down roles over
// the grid (workgroups [0, nb_small) thread per vertex, the next nb_med
// wavefront per vertex, the rest one workgroup per edge chunk) or bottom-up
// word runs over the whole grid.  D is the direction when the launcher
// knows it (host loop: separate top-down and bottom-up instances), or
// kAnyDir to read it from the control block (captured loop).
constexpr int kAnyDir = 2;

// True when the level number is still `seen` (any, if negative) and is the
// launch's (lvl_rem modulo lvl_mod), checked after every earlier load of the
// control block has returned.
__device__ __forceinline__ bool level_still(const Ctl *c, int32_t seen, int32_t lvl_mod, int32_t lvl_rem) {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
  const int32_t lv = __hip_atomic_load(&c->level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (seen < 0 || lv == seen) && lv % lvl_mod == lvl_rem;
}

template <class RowT, int D>
__global__ void __launch_bounds__(1024) k_level(DevG<RowT> G, int32_t nb_small, int32_t nb_med, int32_t mode,
                                                   int32_t lvl_mod, int32_t lvl_rem) {
  const Ctl *c = G.ctl;
  if (c->done) return;
  // This launch is for the level whose number is lvl_rem modulo lvl_mod.
  // Workgroups of a launch can start after its level has been decided (the
  // decide step runs as soon as the workgroups with work have finished); such
  // a workgroup must not act on the next level's state.  So every field is
  // read first and the level number last, once those loads have returned:
  // the decide step writes the number before any other field, so a number
  // that still matches means the fields were read before it ran.
  // (Every workgroup of a bottom-up level takes part in its decide step, so
  // none starts after it; there only the direction read needs the check.)
  const int32_t dir = c->dir;
  if (D != kAnyDir && dir != D) return;
  extern __shared__ __align__(16) char lds[];
  unsigned long long counts[kPartials] = {0, 0, 0, 0};
  unsigned rank = blockIdx.x, nactive = gridDim.x;
  int32_t level;
  if (D == kTD || (D == kAnyDir && dir == kTD)) {
    const TdLevel T = td_level_state(G, c);
    level = T.level;
    if (!level_still(c, T.level, lvl_mod, lvl_rem)) return;
    if (T.from_bitmap) {  // every workgroup takes a share of the frontier words
      const Stage S = stage_open(lds);
      int32_t *ring = reinterpret_cast<int32_t *>(lds + stage_bytes(blockDim.x)) + (threadIdx.x >> 6) * kCandTd;
      unsigned long long tc[2];
      td_level_bitmap(G, T, S, ring, tc);
      counts[0] = tc[0];
      counts[1] = tc[1];
      end_level<kPartials>(G, mode, counts, rank, nactive, T.level);
      return;
    }
    // Only the workgroups whose role has work this level take part: the
    // small and medium roles as many as their queues need (at most nb_small
    // and nb_med; each then covers its queue in one round), the per-chunk
    // role every other workgroup of the grid, up to one per chunk.  The
    // roles take consecutive workgroups in that order.
    const int64_t b = blockIdx.x;
    const int64_t wpb = blockDim.x >> 6;
    const int64_t a_s = min((int64_t)nb_small, (T.cnt[kSmall] + blockDim.x - 1) / blockDim.x);
    const int64_t m_items = T.cnt[kMedium] * medium_split(T.cnt[kMedium], (int64_t)nb_med * wpb, G.t2, T.m_f);
    const int64_t a_m = min((int64_t)nb_med, (m_items + wpb - 1) / wpb);
    const int64_t a_l = min((int64_t)gridDim.x - a_s - a_m, T.nchunk);
    if (b >= a_s + a_m + a_l) return;  // uniform over the workgroup
    rank = (unsigned)b;
    nactive = (unsigned)(a_s + a_m + a_l);
    const Stage S = stage_open(lds);
    unsigned long long tc[2];
    td_level(G, T, S, blockIdx.x, gridDim.x, (int)a_s, (int)a_m, tc);
    counts[0] = tc[0];
    counts[1] = tc[1];
  } else {
    // (dir has been read and used above, so this load follows it; a
    // bottom-up launch of the host loop has no workgroup that starts late)
    level = -1;  // (the decide step reads it)
    if (D == kAnyDir) {
      level = __hip_atomic_load(&c->level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (level % lvl_mod != lvl_rem) return;
    }
    bu_level(G, c, lds, counts);
  }
  end_level<kPartials>(G, mode, counts, rank, nactive, level);
}

// Head records: degree and the first three neighbours (-1 where the row is
// shorter), so short rows and most bottom-up hits need one coalesced 16-byte
// load instead of a row-offset pair and a neighbour-id line.
template <class RowT>
__global__ void k_build_head(const RowT *rp, const int32_t *col, int4 *head, int4 *nb4, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t b = (int64_t)rp[v], e = (int64_t)rp[v + 1];
    const int32_t x0 = b < e ? col[b] : -1, x1 = b + 1 < e ? col[b + 1] : -1, x2 = b + 2 < e ? col[b + 2] : -1;
    head[v] = make_int4((int)(e - b), x0, x1, x2);
    if (nb4) nb4[v] = make_int4(x0, x1, x2, b + 3 < e ? col[b + 3] : -1);  // (rows of at most four)
  }
}

// Compacted head records: the record of the r-th non-isolated vertex (in
// id order) at index r, so a bottom-up level whose candidates are dense
// among the non-isolated vertices reads whole lines of records it uses; and,
// when rpc is not null, the vertex's row offset at the same index (a
// bottom-up level's deferred rows come from consecutive candidates, so their
// offsets share lines).  One thread per 64-vertex word.
template <class RowT>
__global__ void k_build_headc(const int4 *head, const uint64_t *iso, const uint32_t *hrank, const RowT *rp,
                              int4 *headc, uint32_t *rpc, int64_t words) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    uint64_t live = ~iso[w];
    uint32_t r = hrank[w];
    while (live) {
      const int b = __builtin_ctzll(live);
      live &= live - 1;
      headc[r] = head[w * kWave + b];
      if (rpc) rpc[r] = (uint32_t)rp[w * kWave + b];
      ++r;
    }
  }
}

// ---------------------------------------------------------------------------
// Host side.

inline int blocks_for(int64_t items, int64_t per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <class RowT>
DevG<RowT> make_devg(bfs_graph *g) {
  DevG<RowT> G;
  G.rp = static_cast<const RowT *>(g->rp);
  G.col = g->col;
  G.iso = g->iso;
  G.head = g->head;
  G.vis = g->vis;
  for (int s = 0; s < 2; ++s) {
    G.bm[s] = g->bm[s];
    G.sm[s] = g->sm[s];
    G.qs[s] = g->qs[s];
    G.qm[s] = g->qm[s];
    G.ql[s] = g->ql[s];
  }
  G.ctl = g->ctl;
  G.recs = g->recs;
  G.partials = g->partials;
  G.headc = g->headc;
  G.nb4 = g->nb4;
  G.hrank = g->hrank;
  G.rpc = g->rpc;
  G.n = g->n;
  G.words = g->words;
  G.sshift = g->sshift;
  G.swords = (int32_t)g->swords;
  G.t1 = g->params.td_wave_degree;
  G.t2 = g->params.td_block_degree;
  G.tbu = g->params.bu_wave_degree;
  G.td_visited = g->params.td_visited;
  G.qcap = (uint32_t)g->q_cap;
  G.lcap = (uint32_t)g->ql_cap;
  G.slot = g->params.td_visited == BFS_TD_DIST_PLAIN_CULL ? g->slot : nullptr;
  G.pers = 0;
  G.classless = (resolved_policy(g) == BFS_POLICY_TD_ONLY && g->max_degree <= G.t1) ? 1 : 0;
  return G;
}

// Launch shapes shared by both loop drivers.
struct Shapes {
  int bs;            // threads per workgroup
  int wpb;           // wavefronts per workgroup
  int words_blocks;  // one word per wavefront, up to kMaxBlocks workgroups
  int bu_blocks;     // grid of the bottom-up kernel
  size_t lds;        // dynamic LDS of the staging kernels
  size_t level_lds;  // dynamic LDS of the level kernel
};

Shapes shapes_of(const bfs_graph *g) {
  Shapes s;
  s.bs = g->params.block_size;
  s.wpb = s.bs / kWave;
  s.words_blocks = blocks_for(g->words, s.wpb, kMaxBlocks);
  s.bu_blocks = g->params.bu_blocks > 0 ? g->params.bu_blocks : s.words_blocks;
  s.lds = stage_bytes(s.bs);
  const size_t sum_lds = g->sshift >= 0 ? (size_t)g->swords * sizeof(uint64_t) : 0;
  s.level_lds = std::max(s.lds + (size_t)s.wpb * kCandTd * sizeof(int32_t), bu_lds_bytes(s.bs) + sum_lds);
  return s;
}

// Top-down role sizes: at most 512 + 256 + 256 <= kMaxBlocks workgroups.
struct TdRoles {
  int small, med, large;
};

TdRoles td_roles(const Shapes &S, int64_t c0, int64_t c1, int64_t c2, int64_t t2) {
  TdRoles r;
  r.small = c0 > 0 ? blocks_for(c0, S.bs, 512) : 0;
  r.med = c1 > 0 ? blocks_for(c1 * medium_split(1, 1 << 30, t2, INT64_MAX), S.wpb, 256) : 0;  // room to split rows
  r.large = c2 > 0 ? blocks_for(c2, 1, 256) : 0;
  if (r.small + r.med + r.large == 0) r.small = 1;
  return r;
}

template <class RowT>
void launch_level(const DevG<RowT> &G, const Shapes &S, int dir, int blocks, const TdRoles &r, hipStream_t st,
                  int32_t lvl_mod, int32_t lvl_rem) {
  auto *k = dir == kTD ? k_level<RowT, kTD> : dir == kBU ? k_level<RowT, kBU> : k_level<RowT, kAnyDir>;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(S.bs), S.level_lds, st, G, r.small, r.med, (int32_t)kFusedDecide,
                     lvl_mod, lvl_rem);
}

// Level numbers of launches that know their level exactly (host-driven and
// queued loops); captured chunks of K levels check the level modulo K.
constexpr int32_t kExactLevel = 1 << 30;

// Waits for publication number `seq` of a device-driven run (its last
// level).  Sets *published to false when the stream drained without it (the
// captured chunk ended before the search did).
int wait_final(bfs_graph *g, hipStream_t st, uint32_t seq, bool *published) {
  volatile uint32_t *p = &g->ctl_host->seq;
  for (uint64_t spin = 0;; ++spin) {
    if ((int32_t)(__atomic_load_n(p, __ATOMIC_ACQUIRE) - seq) >= 0) {  // (or a later one)
      *published = true;
      return BFS_OK;
    }
    if ((spin & 255) == 255) {
      const hipError_t q = hipStreamQuery(st);
      if (q != hipSuccess && q != hipErrorNotReady)
        return fail(BFS_ERR_DEVICE, "level kernels failed: %s", hipGetErrorString(q));
      if (q == hipSuccess) {
        *published = (int32_t)(__atomic_load_n(p, __ATOMIC_ACQUIRE) - seq) >= 0;
        return BFS_OK;
      }
    }
  }
}

// Waits until the device has published level state number `seq` in the
// host-mapped mirror (polling; the stream is checked now and then so that a
// device error ends the wait), then copies it to *out.
// Copies the mirror once it holds publication `seq` or a later one: the
// copy is retried if the device started another publication meanwhile
// (its number is written before the fields, the completed number after).
int wait_published(bfs_graph *g, hipStream_t st, uint32_t seq, Ctl *out) {
  volatile uint32_t *p = &g->ctl_host->seq;
  volatile uint32_t *wip = &g->ctl_host->seq_wip;
  for (uint64_t spin = 0;; ++spin) {
    const uint32_t got = __atomic_load_n(p, __ATOMIC_ACQUIRE);
    if ((int32_t)(got - seq) >= 0) {
      std::memcpy(out, g->ctl_host, sizeof(Ctl));
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
      if (__atomic_load_n(wip, __ATOMIC_ACQUIRE) == got) {
        out->seq = got;
        return BFS_OK;
      }
      continue;  // torn: a newer publication is being written
    }
    if ((spin & 1023) == 1023) {
      const hipError_t q = hipStreamQuery(st);
      if (q != hipSuccess && q != hipErrorNotReady)
        return fail(BFS_ERR_DEVICE, "level kernels failed: %s", hipGetErrorString(q));
      if (q == hipSuccess && (int32_t)(__atomic_load_n(p, __ATOMIC_ACQUIRE) - seq) < 0)
        return fail(BFS_ERR_DEVICE, "the device did not publish level %u", seq);
    }
  }
}

hipEvent_t level_event(bfs_graph *g, size_t i) {
  while (g->level_events.size() <= i) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g->level_events.push_back(e);
  }
  return g->level_events[i];
}

// Host-driven level loop: after every level the control block is read back,
// so each launch is sized to the frontier it processes.
template <class RowT>
int host_loop(bfs_graph *g, const DevG<RowT> &G, hipStream_t st, std::vector<float> &level_ms) {
  const Shapes S = shapes_of(g);
  const bool timing = g->params.collect_timing != 0;
  int rc;
  size_t nev = 0;
  // Level 0 is known without asking the device: top-down from the source
  // alone (its degree class is not known here, so every role gets a
  // workgroup; the kernel reads the exact counts).  Publication base + 1 is
  // the init kernel's, base + L + 2 the state after level L.
  const uint32_t base = g->pub_seq;
  uint32_t seq = base + 1;
  for (;; ++seq) {
    Ctl h;
    if (seq == base + 1) {
      std::memset(&h, 0, sizeof(h));
      h.dir = kTD;
      h.conv = kConvNone;
      h.qcnt[0][kSmall] = 1;
      h.qcnt[0][kMedium] = 1;
      h.qcnt[0][kLarge] = g->max_degree > G.t2 ? 1 : 0;
      h.qchunk[0] = g->max_degree > G.t2 ? (unsigned)((g->max_degree + G.t2 - 1) / G.t2) : 0;
    } else if ((rc = wait_published(g, st, seq, &h))) {
      return rc;
    }
    if (h.done) break;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {  // the events bracket the level's direction kernel only
      e0 = level_event(g, nev++);
      e1 = level_event(g, nev++);
      if (!e0 || !e1) return fail(BFS_ERR_DEVICE, "hipEventCreate failed");
      BFS_HIP(hipEventRecord(e0, st));
    }
    const int32_t level = seq == base + 1 ? 0 : h.level;
    if (h.dir == kTD && h.conv == kConvB2Q) {  // frontier read from the bitmap, word-parallel
      launch_level(G, S, kTD, S.bu_blocks, TdRoles{0, 0, 0}, st, kExactLevel, level);
    } else if (h.dir == kTD) {
      const TdRoles r = td_roles(S, h.qcnt[h.qcur][0], h.qcnt[h.qcur][1], h.qchunk[h.qcur], G.t2);
      launch_level(G, S, kTD, r.small + r.med + r.large, r, st, kExactLevel, level);
    } else {
      launch_level(G, S, kBU, S.bu_blocks, TdRoles{0, 0, 0}, st, kExactLevel, level);
    }
    if (timing) BFS_HIP(hipEventRecord(e1, st));
    BFS_HIP(hipGetLastError());
  }
  if (timing) {
    // the last level published `done` from inside its kernel, which may
    // still be finishing
    level_ms.clear();
    if (nev > 0) BFS_HIP(hipEventSynchronize(g->level_events[nev - 1]));
    for (size_t i = 0; i + 1 < nev; i += 2) {
      float ms = 0.f;
      BFS_HIP(hipEventElapsedTime(&ms, g->level_events[i], g->level_events[i + 1]));
      level_ms.push_back(ms);
    }
  }
  return BFS_OK;
}

// Captured level loop: `K` levels of fixed-shape launches whose kernels read
// the direction / frontier-form / done flags from the control block; replayed
// until done.
template <class RowT>
int capture_levels(bfs_graph *g, const DevG<RowT> &G, int policy, int K) {
  const Shapes S = shapes_of(g);
  hipStream_t cs = g->cap_stream;
  const bool hybrid = policy != BFS_POLICY_TD_ONLY;
  // fixed role sizes, scaled by graph_td_blocks
  const int gb = g->params.graph_td_blocks;
  TdRoles r;
  r.small = blocks_for(g->n, S.bs, gb);
  r.med = g->max_degree > G.t1 ? blocks_for(g->n, S.wpb, std::max(1, gb / 2)) : 0;
  r.large = g->max_degree > G.t2 ? std::max(1, gb / 2) : 0;
  // one level kernel per level; for hybrid searches its grid serves both
  // directions (extra workgroups join the per-chunk top-down role)
  const int blocks = hybrid ? std::max(r.small + r.med + r.large, S.bu_blocks) : r.small + r.med + r.large;
  release_graph_exec(g);
  BFS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  for (int l = 0; l < K; ++l) {
    launch_level(G, S, kAnyDir, blocks, r, cs, K, l);
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess) return fail(BFS_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  g->graph = graph;
  BFS_HIP(hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0));
  g->gexec_levels = K;
  return BFS_OK;
}

template <class RowT>
int graph_loop(bfs_graph *g, const DevG<RowT> &G, hipStream_t st, int policy) {
  // (at least two levels per chunk: a launch checks its level modulo K)
  const int K = std::max(2, (int)g->params.graph_chunk_levels);
  int rc;
  if (!g->gexec || g->gexec_levels != K) {
    if ((rc = capture_levels(g, G, policy, K))) return rc;
  }
  // the init kernel published number pub_seq + 1, the last level publishes
  // pub_seq + 2; replay the chunk until it has.  Every replay of a running
  // search advances it by K levels; now and then the host makes sure it did.
  const uint32_t target = g->pub_seq + 2;
  int32_t last_level = -1;
  for (int64_t replay = 1;; ++replay) {
    BFS_HIP(hipGraphLaunch(g->gexec, st));
    bool published = false;
    if ((rc = wait_final(g, st, target, &published))) return rc;
    if (published) break;
    if (replay % 64 == 0) {  // the stream has drained: read the level it reached
      Ctl h;
      BFS_HIP(hipMemcpy(&h, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
      if (h.level == last_level || h.done)
        return fail(BFS_ERR_DEVICE,
                    "the captured level loop stopped advancing at level %d (done %d, direction %d, "
                    "queue counts %u/%u/%u, %lld replays)",
                    h.level, h.done, h.dir, h.qcnt[h.qcur][0], h.qcnt[h.qcur][1], h.qcnt[h.qcur][2],
                    (long long)replay);
      last_level = h.level;
    }
  }
  return BFS_OK;
}

// Lookahead loop: the host keeps `ahead` levels enqueued beyond the last
// one the device has published, each as one level kernel with the
// direction read on the device (the kernels of levels past the end exit at
// once), so the device never waits for the host between levels; per-level
// HIP events bracket every level kernel.
template <class RowT>
int queued_loop(bfs_graph *g, const DevG<RowT> &G, hipStream_t st, int policy, std::vector<float> &level_ms) {
  const Shapes S = shapes_of(g);
  const bool hybrid = policy != BFS_POLICY_TD_ONLY;
  const bool timing = g->params.collect_timing != 0;
  const int ahead = g->params.queue_ahead;
  // fixed role sizes, as in the captured loop
  const int gb = g->params.graph_td_blocks;
  TdRoles r;
  r.small = blocks_for(g->n, S.bs, gb);
  r.med = g->max_degree > G.t1 ? blocks_for(g->n, S.wpb, std::max(1, gb / 2)) : 0;
  r.large = g->max_degree > G.t2 ? std::max(1, gb / 2) : 0;
  const int blocks = hybrid ? std::max(r.small + r.med + r.large, S.bu_blocks) : r.small + r.med + r.large;
  const uint32_t base = g->pub_seq;  // init published base + 1, level L publishes base + L + 2
  int enq = 0;
  int rc;
  auto enqueue = [&]() -> int {
    if (timing) {
      hipEvent_t e0 = level_event(g, 2 * (size_t)enq), e1 = level_event(g, 2 * (size_t)enq + 1);
      if (!e0 || !e1) return fail(BFS_ERR_DEVICE, "hipEventCreate failed");
      BFS_HIP(hipEventRecord(e0, st));
      launch_level(G, S, kAnyDir, blocks, r, st, kExactLevel, enq);
      BFS_HIP(hipEventRecord(e1, st));
    } else {
      launch_level(G, S, kAnyDir, blocks, r, st, kExactLevel, enq);
    }
    BFS_HIP(hipGetLastError());
    ++enq;
    return BFS_OK;
  };
  int levels = 0;
  for (int seen = 0;;) {  // seen: the next level whose publication is awaited
    while (enq < seen + ahead)
      if ((rc = enqueue())) return rc;
    Ctl h;
    if ((rc = wait_published(g, st, base + 2 + (uint32_t)seen, &h))) return rc;
    const int level = (int)(h.seq - base - 2);  // the latest published level
    if (h.done) {
      levels = level + 1;
      break;
    }
    seen = level + 1;
  }
  if (timing) {
    level_ms.clear();
    BFS_HIP(hipEventSynchronize(g->level_events[2 * (size_t)levels - 1]));
    for (int l = 0; l < levels; ++l) {
      float ms = 0.f;
      BFS_HIP(hipEventElapsedTime(&ms, g->level_events[2 * l], g->level_events[2 * l + 1]));
      level_ms.push_back(ms);
    }
  }
  return BFS_OK;
}

// Persistent top-down loop: one cooperative launch runs every level.
template <class RowT>
int persistent_loop(bfs_graph *g, const DevG<RowT> &G, hipStream_t st) {
  const Shapes S = shapes_of(g);
  const int nb = g->params.graph_td_blocks;
  int per_cu = 0, cus = 0;
  BFS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_td_persistent<RowT>, S.bs, S.lds));
  BFS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  const int blocks = std::max(1, std::min(nb, per_cu * cus));
  // role split of the fixed grid, by the degree classes the graph has
  // (every class the graph has gets at least one workgroup)
  const int classes = g->max_degree > G.t2 ? 3 : g->max_degree > G.t1 ? 2 : 1;
  if (blocks < classes)
    return fail(BFS_ERR_INVALID_ARG, "graph_td_blocks = %d is below the %d degree classes of this graph",
                blocks, classes);
  const int nb_med = classes >= 2 ? std::max(1, blocks / 4) : 0;
  const int nb_large = classes == 3 ? std::max(1, blocks / 4) : 0;
  const int nb_small = blocks - nb_med - nb_large;
  int32_t a_small = nb_small, a_med = nb_med;
  DevG<RowT> Gp = G;
  Gp.pers = 1;  // levels hand their queues to each other inside the kernel
  void *args[] = {&Gp, &a_small, &a_med};
  BFS_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_td_persistent<RowT>), dim3(blocks),
                                     dim3(S.bs), args, S.lds, st));
  bool published = false;
  int rc = wait_final(g, st, g->pub_seq + 2, &published);
  if (rc) return rc;
  if (!published) return fail(BFS_ERR_DEVICE, "the persistent search ended without publishing its result");
  return BFS_OK;
}

template <class RowT>
int run_impl(bfs_graph *g, int32_t s, int32_t *dist, int32_t *parent) {
  const auto t0 = std::chrono::steady_clock::now();
  const DevG<RowT> G = make_devg<RowT>(g);
  hipStream_t st = g->stream;
  const int policy = resolved_policy(g);
  if (g->params.td_visited != BFS_TD_VISITED_BITMAP && policy != BFS_POLICY_TD_ONLY)
    return fail(BFS_ERR_INVALID_ARG, "td_visited other than the bitmap needs the top-down-only policy");
  for (int q = 0; q < 2; ++q)
    if (!g->qs[q] || !g->qm[q] || !g->ql[q] || g->q_cap < 1 || g->ql_cap < 1)
      return fail(BFS_ERR_OUT_OF_MEMORY, "the frontier queues are not allocated (a failed bfs_set_params?)");
  int loop = g->params.loop;
  if (loop == BFS_LOOP_AUTO) loop = BFS_LOOP_GRAPH;
  if (loop == BFS_LOOP_PERSISTENT && policy != BFS_POLICY_TD_ONLY) loop = BFS_LOOP_HOST;
  const int bs = g->params.block_size;
  g->pub_seq = std::max(g->pub_seq, __atomic_load_n(&g->ctl_host->seq, __ATOMIC_ACQUIRE));
  BFS_HIP(hipEventRecord(g->ev_start, st));
  hipLaunchKernelGGL(k_init<RowT>, dim3(blocks_for(std::max(g->n, g->words), bs, 4096)), dim3(bs), 0, st,
                     G, s, dist, parent, (int32_t)policy, g->params.alpha, g->params.beta, g->nnz,
                     g->rec_cap, g->ctl_host_dev, g->pub_seq,
                     (int32_t)(loop == BFS_LOOP_HOST || loop == BFS_LOOP_QUEUED ? kPubEvery : kPubFinal));
  BFS_HIP(hipGetLastError());
  std::vector<float> level_ms;
  int rc = loop == BFS_LOOP_HOST    ? host_loop(g, G, st, level_ms)
           : loop == BFS_LOOP_GRAPH ? graph_loop(g, G, st, policy)
           : loop == BFS_LOOP_QUEUED ? queued_loop(g, G, st, policy, level_ms)
                                    : persistent_loop(g, G, st);
  if (rc) {
    g->pub_seq += 1u << 20;  // keep later runs clear of anything this run may still publish
    return rc;
  }
  BFS_HIP(hipEventRecord(g->ev_stop, st));
  BFS_HIP(hipEventSynchronize(g->ev_stop));
  const auto t1 = std::chrono::steady_clock::now();
  float dev_ms = 0.f;
  BFS_HIP(hipEventElapsedTime(&dev_ms, g->ev_start, g->ev_stop));
  const Ctl h = *g->ctl_host;  // final state (read by the loop after the last level)
  g->pub_seq = h.seq;
  const int nrec = std::min(h.levels_done, g->rec_cap);
  std::vector<LevelRec> recs(nrec);
  if (nrec > 0)
    BFS_HIP(hipMemcpy(recs.data(), g->recs, sizeof(LevelRec) * nrec, hipMemcpyDeviceToHost));
  g->last_levels.resize(nrec);
  for (int i = 0; i < nrec; ++i) {
    bfs_level_stats &o = g->last_levels[i];
    const LevelRec &r = recs[i];
    o.level = r.level;
    o.direction = r.dir;
    o.frontier = r.n_f;
    o.frontier_edges = r.m_f;
    o.unvisited_edges = r.m_u;
    o.discovered = r.found;
    o.scanned = r.scanned;
    o.examined = r.examined;
    o.ms = i < (int)level_ms.size() ? level_ms[i] : 0.f;
    o.pad = 0.f;
  }
  bfs_run_stats &L = g->last;
  L.source = s;
  L.levels = h.levels_done;
  L.reached = h.reached;
  L.edges = h.sum_mf / 2;
  L.device_ms = dev_ms;
  L.host_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  L.loop = loop;
  L.policy = policy;
  if (h.overflow == 2)
    return fail(BFS_ERR_DEVICE, "the persistent search stopped at level %d: a workgroup waited more than "
                                "%llu polls for the level to end", h.levels_done,
                (unsigned long long)kPersistSpinLimit);
  if (h.overflow)
    return fail(BFS_ERR_OUT_OF_MEMORY,
                "level %d appended more frontier entries than the queues hold (%lld per small/medium "
                "queue, %lld per large queue); distances past that level are incomplete",
                h.levels_done - 1, (long long)g->q_cap, (long long)g->ql_cap);
  return BFS_OK;
}

}  // namespace

int build_head(bfs_graph *g) {
  const int bs = 256;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + bs - 1) / bs, 8192));
  if (g->rp64)
    hipLaunchKernelGGL(k_build_head<int64_t>, dim3(blocks), dim3(bs), 0, nullptr,
                       static_cast<const int64_t *>(g->rp), g->col, g->head, g->nb4, g->n);
  else
    hipLaunchKernelGGL(k_build_head<int32_t>, dim3(blocks), dim3(bs), 0, nullptr,
                       static_cast<const int32_t *>(g->rp), g->col, g->head, g->nb4, g->n);
  if (g->rp64)
    hipLaunchKernelGGL(k_build_headc<int64_t>, dim3(blocks), dim3(bs), 0, nullptr, g->head, g->iso, g->hrank,
                       static_cast<const int64_t *>(g->rp), g->headc, g->rpc, g->words);
  else
    hipLaunchKernelGGL(k_build_headc<int32_t>, dim3(blocks), dim3(bs), 0, nullptr, g->head, g->iso, g->hrank,
                       static_cast<const int32_t *>(g->rp), g->headc, g->rpc, g->words);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipDeviceSynchronize());
  return BFS_OK;
}

int run_single(bfs_graph *g, int32_t source, int32_t *dist, int32_t *parent) {
  return g->rp64 ? run_impl<int64_t>(g, source, dist, parent) : run_impl<int32_t>(g, source, dist, parent);
}

}  // namespace bfsmi
