// Serving: continuous batching of single-source BFS requests.
//
// Requests for one graph run together as lanes of a multi-source search (up
// to 64 lanes, one bit per lane in 64-bit per-vertex sets, as in the batched
// search).  A request joins a running batch at the next chunk boundary
// (every few levels) when a lane is free, and retires as soon as its own
// frontier is empty, so lanes of one batch start and finish at different
// levels.  Each lane writes int32 distances counted from the level at which
// it joined (and, when asked, parents) into the caller's buffers, so a
// request's result does not depend on which other requests share its
// batch.  Batches of different graphs (or several of one graph) run on
// their own streams and overlap on the device; a background thread admits
// queued requests when a lane and the memory budget allow.
//
// Per level (all kernels read the level state from the batch's control
// block, so a whole chunk of levels is issued without host round trips):
//   expand    top-down: the frontier queue's vertices push their lane sets
//             to unseen neighbours (atomicOr into next[x]; the first pusher
//             of x appends it to the touched list); bottom-up: every vertex
//             with unfinished live lanes gathers its neighbours' frontier
//             sets, stopping once all its missing lanes are found.  The
//             frontier sets alternate between two arrays by level parity;
//             expand also clears, in the other array, the sets of the
//             previous level's frontier (that array receives the next
//             frontier);
//   finalize  touched vertices: new lanes become seen and frontier, their
//             distances are written, the vertex joins the next frontier
//             queue; the last workgroup reduces the level's counts and picks
//             the next direction (the decide step).
// Top-down levels touch only the frontier and its edges, so large-diameter
// graphs cost per level what their frontier costs.

#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

#include "common.h"
#include "device_util.h"

namespace bfsmi {
namespace {

constexpr int kLanes = 64;
constexpr int kSvMaxBlocks = 1024;
// Top-down rows longer than kSvChunk edges are expanded as kSvChunk-edge
// chunks spread over every wavefront of the grid (a hub's row walked by one
// wavefront would take one dependent step per 64 edges: tens of
// milliseconds for a million-edge hub).
constexpr int64_t kSvChunk = 512;

struct alignas(256) ServeCtl {
  int32_t dir;    // direction of the next level (0 top-down, 1 bottom-up)
  int32_t level;  // next batch level to run
  int32_t fsel;   // frontier queue holding the current frontier
  int32_t pad0;
  unsigned int fcnt[2];  // entries in frontier queue 0 / 1
  unsigned int tcnt;     // entries in the touched list of the running level
  unsigned int pad1;
  unsigned long long alive;        // lanes whose frontier is not empty
  unsigned long long join_mask;    // lanes (re)initialised at this boundary
  unsigned long long parent_mask;  // lanes that record parents
  int32_t start[kLanes];     // batch level at which each lane joined
  int32_t finish[kLanes];    // batch level after the lane's last level
  int32_t join_src[kLanes];  // sources of the joining lanes
  int32_t *dist[kLanes];
  int32_t *parent[kLanes];
  int32_t levels_run;
  int32_t bu_percent;
  unsigned int hcnt[2];  // entries in chunk queue 0 / 1 (rows longer than kSvChunk)
  unsigned int pcnt;     // entries of the previous level's frontier (queue fsel ^ 1)
};

template <class RowT>
struct SvArgs {
  const RowT *rp;
  const int32_t *col;
  int64_t n, nnz;
  uint64_t *seen, *next;
  uint64_t *fr[2];  // frontier sets of even / odd batch levels
  int32_t *fq[2];  // frontier queues
  uint64_t *hq[2];  // chunk queues of the long rows of each frontier: chunk << 32 | v
  int64_t hq_cap;
  int32_t *tq;     // touched list
  unsigned long long *partials;  // [kSvMaxBlocks][3]
  ServeCtl *ctl;
};

// Single-bucket workgroup staging of vertex ids in LDS (capacity 4 per
// thread), copied out with one global atomicAdd per workgroup; slots past
// the capacity go straight to the global list.
struct Stage1 {
  unsigned *cnt;
  int32_t *buf;
  unsigned cap;
};

__host__ __device__ constexpr size_t stage1_bytes(int bs) { return 16 + (size_t)16 * bs; }

__device__ __forceinline__ Stage1 stage1_open(char *lds) {
  Stage1 S;
  S.cnt = reinterpret_cast<unsigned *>(lds);
  S.buf = reinterpret_cast<int32_t *>(lds + 16);
  S.cap = 4 * blockDim.x;
  if (threadIdx.x == 0) *S.cnt = 0;
  __syncthreads();
  return S;
}

// All lanes of a wavefront call together.
__device__ __forceinline__ void stage1_push(const Stage1 &S, bool p, int32_t v, int32_t *gq,
                                            unsigned *gcnt) {
  const uint64_t m = __ballot(p);
  if (!m) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  const unsigned k = (unsigned)__popcll(m);
  unsigned base = 0;
  if (lane_id() == leader) base = atomicAdd(S.cnt, k);
  base = __shfl(base, leader);
  const unsigned first_over = base > S.cap ? base : S.cap;
  const unsigned over = base + k > S.cap ? base + k - first_over : 0;
  unsigned gbase = 0;
  if (over) {
    if (lane_id() == leader) gbase = atomicAdd(gcnt, over);
    gbase = __shfl(gbase, leader);
  }
  if (p) {
    const unsigned slot = base + lanes_below(m);
    if (slot < S.cap)
      S.buf[slot] = v;
    else
      gq[gbase + (slot - first_over)] = v;
  }
}

// Appends the kSvChunk-edge chunks of frontier vertex v (degree deg) to
// chunk queue `sel`.  The queue holds every chunk of one level: each of its
// vertices has degree > kSvChunk, so a level has fewer than 2 nnz / kSvChunk
// chunks; entries past hq_cap are never written.
template <class RowT>
__device__ __forceinline__ void push_chunks(const SvArgs<RowT> &A, ServeCtl *c, int sel, int32_t v, int64_t deg) {
  const unsigned nch = (unsigned)((deg + kSvChunk - 1) / kSvChunk);
  const unsigned base = atomicAdd(&c->hcnt[sel], nch);
  uint64_t *hq = sel ? A.hq[1] : A.hq[0];
  for (unsigned k = 0; k < nch; ++k)
    if ((int64_t)(base + k) < A.hq_cap) hq[base + k] = ((uint64_t)k << 32) | (uint32_t)v;
}

// All threads of the workgroup call.
__device__ __forceinline__ void stage1_flush(const Stage1 &S, int32_t *gq, unsigned *gcnt) {
  __shared__ unsigned gbase, count;
  __syncthreads();
  if (threadIdx.x == 0) {
    count = *S.cnt < S.cap ? *S.cnt : S.cap;
    gbase = count ? atomicAdd(gcnt, count) : 0;
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < count; i += blockDim.x) gq[gbase + i] = S.buf[i];
}

// Joining lanes: clear their bits left in `seen` by earlier occupants, and
// initialise their outputs (dist = -1, parent = -1).
template <class RowT>
__global__ void k_sv_join(SvArgs<RowT> A) {
  const ServeCtl *c = A.ctl;
  const unsigned long long m = c->join_mask;
  if (!m) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < A.n; v += stride) {
    const uint64_t s = A.seen[v];
    if (s & m) A.seen[v] = s & ~m;
    uint64_t b = m;
    while (b) {
      const int i = __ffsll((unsigned long long)b) - 1;
      b &= b - 1;
      // (streaming stores: output rows, never read by the server)
      __builtin_nontemporal_store(-1, c->dist[i] + v);
      if (c->parent[i]) __builtin_nontemporal_store(-1, c->parent[i] + v);
    }
  }
}

// Joining lanes: mark their sources (one workgroup of 64 threads).
template <class RowT>
__global__ void k_sv_seed(SvArgs<RowT> A) {
  ServeCtl *c = A.ctl;
  const unsigned long long m = c->join_mask;
  const int i = threadIdx.x;
  if ((m >> i) & 1ull) {
    const int32_t s = c->join_src[i];
    const unsigned long long bit = 1ull << i;
    atomicOr(reinterpret_cast<unsigned long long *>(A.seen + s), bit);
    const unsigned long long old = atomicOr(reinterpret_cast<unsigned long long *>(A.fr[c->level & 1] + s), bit);
    if (old == 0) {  // s is not on the frontier yet: append it once
      const unsigned slot = atomicAdd(&c->fcnt[c->fsel], 1u);
      A.fq[c->fsel][slot] = s;
      const int64_t deg = (int64_t)A.rp[s + 1] - (int64_t)A.rp[s];
      if (deg > kSvChunk) push_chunks(A, c, c->fsel, s, deg);
    }
    c->dist[i][s] = 0;
    if (c->parent[i]) c->parent[i][s] = s;
    c->start[i] = c->level;
  }
  __syncthreads();
  if (i == 0 && m) {
    c->alive |= m;
    c->join_mask = 0;
  }
}

// Records parent u for the lanes in `bits` of vertex x.
__device__ __forceinline__ void write_parents(const ServeCtl *c, uint64_t bits, int64_t x, int32_t u) {
  while (bits) {
    const int i = __ffsll((unsigned long long)bits) - 1;
    bits &= bits - 1;
    __builtin_nontemporal_store(u, c->parent[i] + x);
  }
}

template <class RowT>
__global__ void k_sv_expand(SvArgs<RowT> A) {
  const ServeCtl *c = A.ctl;
  const uint64_t alive = c->alive;
  if (!alive) return;
  extern __shared__ __align__(16) char lds[];
  const Stage1 S = stage1_open(lds);
  ServeCtl *cw = A.ctl;
  const uint64_t pmask = c->parent_mask;
  const int lane = lane_id();
  const int64_t wpb = blockDim.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * wpb;
  const int64_t gw = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const uint64_t *front = A.fr[c->level & 1];
  {  // the previous frontier's sets, in the array the next frontier goes to
    uint64_t *stale = A.fr[(c->level & 1) ^ 1];
    const int32_t *pq = c->fsel ? A.fq[0] : A.fq[1];
    const int64_t np = c->pcnt;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) stale[pq[i]] = 0;
  }
  if (c->dir == 0) {
    // Top-down over the frontier queue, 64 entries per wavefront step.
    const int32_t *fq = c->fsel ? A.fq[1] : A.fq[0];
    const int64_t nf = c->fcnt[c->fsel];
    for (int64_t base = gw * kWave; base < nf; base += nwaves * kWave) {
      const int64_t i = base + lane;
      int32_t v = i < nf ? fq[i] : -1;
      uint64_t f = 0;
      int64_t beg = 0, end = 0;
      if (v >= 0) {
        beg = (int64_t)A.rp[v];
        end = (int64_t)A.rp[v + 1];
        if (end - beg > kSvChunk) {  // a long row: its chunks are expanded below
          v = -1;
          beg = end = 0;
        } else {
          f = front[v];
        }
      }
      const bool heavy = (end - beg) > kWave;
      bool any_push = false;
      if (!heavy) {
        for (int64_t j = beg; __ballot(j < end); ++j) {
          const bool has = j < end;
          int32_t x = 0;
          bool first = false;
          if (has) {
            x = A.col[j];
            const uint64_t nb = f & ~A.seen[x];
            if (nb) {
              const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), nb);
              first = (old == 0);
              if (nb & pmask & ~old) write_parents(c, nb & pmask & ~old, x, v);
            }
          }
          stage1_push(S, first, x, A.tq, &cw->tcnt);
          any_push |= first;
        }
      }
      uint64_t hm = __ballot(heavy);
      while (hm) {
        const int l = __ffsll((unsigned long long)hm) - 1;
        hm &= hm - 1;
        const int64_t b0 = __shfl(beg, l), e0 = __shfl(end, l);
        const uint64_t fl = __shfl(f, l);
        const int32_t vl = __shfl(v, l);
        for (int64_t b = b0; b < e0; b += kWave) {
          const int64_t j = b + lane;
          int32_t x = 0;
          bool first = false;
          if (j < e0) {
            x = A.col[j];
            const uint64_t nb = fl & ~A.seen[x];
            if (nb) {
              const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), nb);
              first = (old == 0);
              if (nb & pmask & ~old) write_parents(c, nb & pmask & ~old, x, vl);
            }
          }
          stage1_push(S, first, x, A.tq, &cw->tcnt);
        }
      }
      (void)any_push;
    }
    // the long rows, one kSvChunk-edge chunk per wavefront
    const uint64_t *hq = c->fsel ? A.hq[1] : A.hq[0];
    const int64_t nh = min((int64_t)c->hcnt[c->fsel], A.hq_cap);
    for (int64_t i = gw; i < nh; i += nwaves) {
      const uint64_t e = hq[i];
      const int32_t vl = (int32_t)(uint32_t)e;
      const uint64_t fl = front[vl];
      const int64_t b0 = (int64_t)A.rp[vl] + (int64_t)(e >> 32) * kSvChunk;
      const int64_t e0 = min((int64_t)A.rp[vl + 1], b0 + kSvChunk);
      for (int64_t b = b0; b < e0; b += kWave) {
        const int64_t j = b + lane;
        int32_t x = 0;
        bool first = false;
        if (j < e0) {
          x = A.col[j];
          const uint64_t nb = fl & ~A.seen[x];
          if (nb) {
            const uint64_t old = atomicOr(reinterpret_cast<unsigned long long *>(A.next + x), nb);
            first = (old == 0);
            if (nb & pmask & ~old) write_parents(c, nb & pmask & ~old, x, vl);
          }
        }
        stage1_push(S, first, x, A.tq, &cw->tcnt);
      }
    }
  } else {
    // Bottom-up over all vertices, one 64-vertex group per wavefront step.
    const int64_t groups = (A.n + kWave - 1) / kWave;
    for (int64_t gi = gw; gi < groups; gi += nwaves) {
      const int64_t v = gi * kWave + lane;
      const uint64_t target = v < A.n ? (~A.seen[v] & alive) : 0ull;
      int64_t beg = 0, end = 0;
      if (target) {
        beg = (int64_t)A.rp[v];
        end = (int64_t)A.rp[v + 1];
      }
      const bool heavy = (end - beg) > kWave;
      uint64_t acc = 0;
      if (target && !heavy) {
        for (int64_t j = beg; j < end; ++j) {
          const int32_t x = A.col[j];
          const uint64_t fr = front[x] & target & ~acc;
          if (fr) {
            if (fr & pmask) write_parents(c, fr & pmask, v, x);
            acc |= fr;
            if (acc == target) break;
          }
        }
      }
      uint64_t hm = __ballot(heavy);
      while (hm) {
        const int l = __ffsll((unsigned long long)hm) - 1;
        hm &= hm - 1;
        const int64_t b0 = __shfl(beg, l), e0 = __shfl(end, l);
        const uint64_t tl = __shfl(target, l);
        const int64_t vl = __shfl(v, l);
        uint64_t al = 0;
        for (int64_t b = b0; b < e0; b += kWave) {
          const int64_t j = b + lane;
          const int32_t x = j < e0 ? A.col[j] : 0;
          const uint64_t fr = j < e0 ? (front[x] & tl) : 0ull;
          uint64_t fresh = wave_or(fr) & ~al;
          if (fresh & pmask) {  // parent of each new lane: its lowest contributing position
            uint64_t pb = fresh & pmask;
            while (pb) {
              const int i = __ffsll((unsigned long long)pb) - 1;
              pb &= pb - 1;
              const uint64_t who = __ballot((fr >> i) & 1ull);
              const int src = __ffsll((unsigned long long)who) - 1;
              const int32_t px = __shfl(x, src);
              if (lane == 0) __builtin_nontemporal_store(px, c->parent[i] + vl);
            }
          }
          al |= fresh;
          if (al == tl) break;
        }
        if (lane == l) acc = al;
      }
      const bool got = acc != 0;
      if (got) A.next[v] = acc;
      stage1_push(S, got, (int32_t)v, A.tq, &cw->tcnt);
    }
  }
  stage1_flush(S, A.tq, &cw->tcnt);
}

// Touched vertices become the new frontier.
// Accumulators of the level's totals (new lane pairs, frontier edges, OR of
// the new lanes) per group of workgroups, then the groups' arrival counters
// and the counter over the groups, each in its own 128-byte line of the
// batch's partials array.
constexpr int kSvGroups = 8;
constexpr int kSvLine = 16;  // 64-bit words per 128-byte line
constexpr size_t kSvArriveOffset = (size_t)kSvGroups * 3 * kSvLine;
static_assert(kSvArriveOffset + (kSvGroups + 1) * kSvLine <= (size_t)kSvMaxBlocks * 3,
              "the partials array holds the accumulators and counters");

// Touched vertices become the new frontier; the last workgroup to finish
// then reduces the level's totals and applies the decide step (lanes whose
// frontier emptied finish, the direction of the next level).  Only the
// workgroups that have touched entries take part, and workgroup 0 always
// does, so no workgroup can start after the decide step and act on the next
// level (the reset touched count makes every workgroup but 0 idle).
template <class RowT>
__global__ void k_sv_finalize(SvArgs<RowT> A) {
  ServeCtl *c = A.ctl;
  if (!c->alive) return;
  const int64_t nt = c->tcnt;
  const int64_t nact = max((int64_t)1, min((int64_t)gridDim.x, (nt + blockDim.x - 1) / blockDim.x));
  if ((int64_t)blockIdx.x >= nact) return;  // uniform: no touched entry for this workgroup
  extern __shared__ __align__(16) char lds[];
  const Stage1 S = stage1_open(lds);
  const int nsel = c->fsel ^ 1;
  int32_t *fq_next = nsel ? A.fq[1] : A.fq[0];
  unsigned *fcnt_next = &c->fcnt[nsel];
  const int32_t level = c->level;
  unsigned long long pairs = 0, fedges = 0, bits = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole wavefronts step together (stage1_push is a wavefront operation)
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < nt; base += stride) {
    const int64_t i = base + lane_id();
    uint64_t nb = 0;
    int32_t x = 0;
    if (i < nt) {
      x = A.tq[i];
      const uint64_t s = A.seen[x];
      nb = A.next[x] & ~s;
      A.next[x] = 0;
      A.fr[(level & 1) ^ 1][x] = nb;
      if (nb) {
        A.seen[x] = s | nb;
        pairs += (unsigned long long)__popcll(nb);
        const int64_t deg = (int64_t)A.rp[x + 1] - (int64_t)A.rp[x];
        fedges += (unsigned long long)deg;
        if (deg > kSvChunk) push_chunks(A, c, nsel, x, deg);
        bits |= nb;
        uint64_t b = nb;
        while (b) {
          const int k = __ffsll((unsigned long long)b) - 1;
          b &= b - 1;
          __builtin_nontemporal_store(level + 1 - c->start[k], c->dist[k] + x);
        }
      }
    }
    stage1_push(S, nb != 0, x, fq_next, fcnt_next);
  }
  stage1_flush(S, fq_next, fcnt_next);
  __shared__ unsigned long long part[3][16];
  pairs = wave_sum(pairs);
  fedges = wave_sum(fedges);
  bits = wave_or(bits);
  if (lane_id() == 0) {
    part[0][threadIdx.x >> 6] = pairs;
    part[1][threadIdx.x >> 6] = fedges;
    part[2][threadIdx.x >> 6] = bits;
  }
  __syncthreads();
  if (threadIdx.x >= kWave) return;  // wave 0 finishes
  const int lane = threadIdx.x;
  unsigned long long t = 0;
  if (lane < 3)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = lane == 2 ? (t | part[2][w]) : t + part[lane][w];
  unsigned long long *acc = A.partials;
  unsigned long long *arrive = A.partials + kSvArriveOffset;
  const unsigned grp = blockIdx.x % kSvGroups;
  const unsigned na = (unsigned)nact;
  const unsigned gsize = (na - grp + kSvGroups - 1) / kSvGroups;
  const unsigned ngroups = na < (unsigned)kSvGroups ? na : (unsigned)kSvGroups;
  if (lane < 3 && t) {
    unsigned long long *a = acc + ((size_t)grp * 3 + lane) * kSvLine;
    if (lane == 2) atomicOr(a, t);
    else atomicAdd(a, t);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the adds complete before the arrival
  unsigned long long arrived = 0;
  if (gsize > 1) {
    if (lane == 0) arrived = atomicAdd(arrive + (size_t)grp * kSvLine, 1ull);
    if (__shfl(arrived, 0) != gsize - 1) return;
    if (lane == 0) atomicExch(arrive + (size_t)grp * kSvLine, 0ull);
  }
  if (lane == 0) arrived = atomicAdd(arrive + (size_t)kSvGroups * kSvLine, 1ull);
  if (__shfl(arrived, 0) != ngroups - 1) return;
  if (lane == 0) atomicExch(arrive + (size_t)kSvGroups * kSvLine, 0ull);
  // lane g * 3 + k takes accumulator k of group g
  unsigned long long x = 0;
  if ((unsigned)lane < ngroups * 3) x = atomicExch(acc + (size_t)lane * kSvLine, 0ull);
  unsigned long long tf = 0, tb = 0;
  for (unsigned g = 0; g < ngroups; ++g) {
    tf += __shfl(x, (int)(g * 3 + 1));
    tb |= __shfl(x, (int)(g * 3 + 2));
  }
  if (lane != 0) return;
  uint64_t ended = c->alive & ~tb;  // lanes whose new frontier is empty
  while (ended) {
    const int i = __ffsll((unsigned long long)ended) - 1;
    ended &= ended - 1;
    c->finish[i] = level + 1;
  }
  c->alive = tb;
  c->pcnt = c->fcnt[c->fsel];
  c->fcnt[c->fsel] = 0;
  c->hcnt[c->fsel] = 0;
  c->fsel ^= 1;
  c->tcnt = 0;
  c->level = level + 1;
  c->levels_run += 1;
  c->dir = (tf * 100ull > (unsigned long long)c->bu_percent * (unsigned long long)A.nnz) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Host side.

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  bfs_graph *g = nullptr;
  int32_t source = 0;
  int32_t *dist = nullptr;
  int32_t *parent = nullptr;
  int32_t state = BFS_REQ_QUEUED;
  int32_t lanes_at_admit = 0;
  int32_t start_level = 0;
  int32_t levels = 0;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
};

struct Batch {
  bfs_graph *g = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  uint64_t *seen = nullptr, *fr[2] = {nullptr, nullptr}, *next = nullptr;
  int32_t *fq[2] = {nullptr, nullptr};
  uint64_t *hq[2] = {nullptr, nullptr};
  int64_t hq_cap = 0;
  int32_t *tq = nullptr;
  unsigned long long *partials = nullptr;
  ServeCtl *ctl = nullptr;       // device
  ServeCtl *mirror = nullptr;    // pinned host copy
  Request *lane[kLanes] = {};
  uint64_t active = 0;
  bool in_flight = false;
  size_t bytes = 0;
};

// Chunk entries one level can hold: every chunked row has more than
// kSvChunk edges, so its chunks number under 2 deg / kSvChunk.
int64_t chunk_capacity(const bfs_graph *g) { return 2 * (g->nnz / kSvChunk) + 2 * kLanes; }

size_t batch_bytes(const bfs_graph *g) {
  return (size_t)g->n * (4 * 8 + 3 * 4) + 2 * sizeof(uint64_t) * (size_t)chunk_capacity(g) +
         sizeof(unsigned long long) * kSvMaxBlocks * 3 + sizeof(ServeCtl);
}

}  // namespace
}  // namespace bfsmi

struct bfs_server {
  size_t budget = 0;
  int max_lanes = 64;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::deque<bfsmi::Request *> inbox;                        // submitted, not yet seen by the worker
  std::map<bfs_graph *, std::deque<bfsmi::Request *>> waiting;  // per graph, in arrival order
  std::unordered_map<uint64_t, std::unique_ptr<bfsmi::Request>> reqs;
  std::vector<std::unique_ptr<bfsmi::Batch>> batches;
  size_t used = 0;
  uint64_t next_ticket = 1;
  std::string worker_error;
};

namespace bfsmi {
namespace {

void free_batch(Batch *b) {
  DeviceGuard dg(b->g->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  void *ptrs[] = {b->seen, b->fr[0], b->fr[1], b->next, b->fq[0], b->fq[1], b->hq[0], b->hq[1], b->tq,
                  b->partials, b->ctl};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (b->mirror) (void)hipHostFree(b->mirror);
  if (b->ev) (void)hipEventDestroy(b->ev);
  if (b->stream) (void)hipStreamDestroy(b->stream);
}

// Allocates and clears a batch's device state; false on failure.
bool make_batch(Batch *b, bfs_graph *g) {
  DeviceGuard dg(g->device);
  b->g = g;
  const size_t n = (size_t)g->n;
  bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) == hipSuccess;
  b->hq_cap = chunk_capacity(g);
  void **dst[] = {(void **)&b->seen, (void **)&b->fr[0], (void **)&b->next, (void **)&b->fq[0],
                  (void **)&b->fq[1], (void **)&b->tq, (void **)&b->partials, (void **)&b->ctl,
                  (void **)&b->hq[0], (void **)&b->hq[1], (void **)&b->fr[1]};
  const size_t sizes[] = {8 * n, 8 * n, 8 * n, 4 * n, 4 * n, 4 * n,
                          sizeof(unsigned long long) * kSvMaxBlocks * 3, sizeof(ServeCtl),
                          sizeof(uint64_t) * (size_t)b->hq_cap, sizeof(uint64_t) * (size_t)b->hq_cap, 8 * n};
  for (int i = 0; i < 11 && ok; ++i) ok = hipMalloc(dst[i], std::max<size_t>(sizes[i], 8)) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&b->mirror, sizeof(ServeCtl), hipHostMallocDefault) == hipSuccess;
  if (ok) {
    ok = hipMemsetAsync(b->seen, 0, 8 * n, b->stream) == hipSuccess &&
         hipMemsetAsync(b->fr[0], 0, 8 * n, b->stream) == hipSuccess &&
         hipMemsetAsync(b->fr[1], 0, 8 * n, b->stream) == hipSuccess &&
         hipMemsetAsync(b->next, 0, 8 * n, b->stream) == hipSuccess &&
         hipMemsetAsync(b->partials, 0, sizes[6], b->stream) == hipSuccess;
    std::memset(b->mirror, 0, sizeof(ServeCtl));
    b->mirror->bu_percent = g->params.msbfs_bu_percent;
  }
  b->bytes = batch_bytes(g);
  return ok;
}

template <class RowT>
SvArgs<RowT> args_of(Batch *b) {
  SvArgs<RowT> A;
  A.rp = static_cast<const RowT *>(b->g->rp);
  A.col = b->g->col;
  A.n = b->g->n;
  A.nnz = b->g->nnz;
  A.seen = b->seen;
  A.fr[0] = b->fr[0];
  A.fr[1] = b->fr[1];
  A.next = b->next;
  A.fq[0] = b->fq[0];
  A.fq[1] = b->fq[1];
  A.hq[0] = b->hq[0];
  A.hq[1] = b->hq[1];
  A.hq_cap = b->hq_cap;
  A.tq = b->tq;
  A.partials = b->partials;
  A.ctl = b->ctl;
  return A;
}

// Issues: control block upload, lane joins, `levels` levels, control block
// download, completion event.
template <class RowT>
int issue_chunk(Batch *b, int levels) {
  const SvArgs<RowT> A = args_of<RowT>(b);
  hipStream_t st = b->stream;
  const int bs = 512;
  const int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(kSvMaxBlocks, (b->g->n + bs - 1) / bs));
  const size_t lds = stage1_bytes(bs);
  BFS_HIP(hipMemcpyAsync(b->ctl, b->mirror, sizeof(ServeCtl), hipMemcpyHostToDevice, st));
  if (b->mirror->join_mask) {
    hipLaunchKernelGGL(k_sv_join<RowT>, dim3(nblocks), dim3(bs), 0, st, A);
    hipLaunchKernelGGL(k_sv_seed<RowT>, dim3(1), dim3(kLanes), 0, st, A);
  }
  for (int l = 0; l < levels; ++l) {
    hipLaunchKernelGGL(k_sv_expand<RowT>, dim3(nblocks), dim3(bs), lds, st, A);
    hipLaunchKernelGGL(k_sv_finalize<RowT>, dim3(nblocks), dim3(bs), lds, st, A);
  }
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipMemcpyAsync(b->mirror, b->ctl, sizeof(ServeCtl), hipMemcpyDeviceToHost, st));
  BFS_HIP(hipEventRecord(b->ev, st));
  b->in_flight = true;
  return BFS_OK;
}

// Levels per issued chunk.  Large-diameter graphs run long chunks (their
// levels are many and cheap, and every chunk boundary is a host round trip),
// but only while no other batch is active and no other graph's request
// waits: the streams of different batches share the device's few hardware
// queues, and a chunk of a thousands-of-levels search ahead of another
// batch's kernels would hold those back for its whole length.
constexpr int kSvSharedChunk = 8;
int chunk_levels(const bfs_graph *g, bool shared) {
  if (g->nnz < 7 * g->n) return shared ? kSvSharedChunk : 32;  // large-diameter class
  return 4;
}

}  // namespace
}  // namespace bfsmi

using namespace bfsmi;

namespace {

// Fills free lanes of an idle batch from its graph's waiting queue.
void admit(bfs_server *s, Batch *b) {
  auto it = s->waiting.find(b->g);
  if (it == s->waiting.end()) return;
  auto &q = it->second;
  ServeCtl *m = b->mirror;
  while (!q.empty() && __builtin_popcountll(b->active) < s->max_lanes) {
    const int i = __builtin_ctzll(~b->active);
    Request *r = q.front();
    q.pop_front();
    b->lane[i] = r;
    b->active |= 1ull << i;
    m->join_mask |= 1ull << i;
    m->join_src[i] = r->source;
    m->dist[i] = r->dist;
    m->parent[i] = r->parent;
    if (r->parent)
      m->parent_mask |= 1ull << i;
    else
      m->parent_mask &= ~(1ull << i);
    r->state = BFS_REQ_RUNNING;
    r->t_admit = now_ns();
    r->start_level = m->level;
  }
  for (int i = 0; i < kLanes; ++i)
    if ((m->join_mask >> i) & 1ull) b->lane[i]->lanes_at_admit = __builtin_popcountll(b->active);
  if (q.empty()) s->waiting.erase(it);
}

// Retires the lanes whose frontier emptied during the finished chunk.
void retire(bfs_server *s, Batch *b) {
  const uint64_t done = b->active & ~b->mirror->alive;
  const int64_t t = now_ns();
  for (int i = 0; i < kLanes; ++i) {
    if (!((done >> i) & 1ull)) continue;
    Request *r = b->lane[i];
    r->levels = b->mirror->finish[i] - b->mirror->start[i];
    r->t_done = t;
    r->state = BFS_REQ_DONE;
    r->g->server_refs.fetch_sub(1);
    b->lane[i] = nullptr;
  }
  b->active &= ~done;
}

void fail_batch(bfs_server *s, Batch *b, const char *why) {
  for (int i = 0; i < kLanes; ++i) {
    if (!b->lane[i]) continue;
    b->lane[i]->state = BFS_REQ_FAILED;
    b->lane[i]->t_done = now_ns();
    b->lane[i]->g->server_refs.fetch_sub(1);
    b->lane[i] = nullptr;
  }
  b->active = 0;
  s->worker_error = why;
}

// True when a batch of g has a free lane.
bool has_room(const bfs_server *s, const bfs_graph *g) {
  for (const auto &b : s->batches)
    if (b->g == g && __builtin_popcountll(b->active) < s->max_lanes) return true;
  return false;
}

// Frees empty, idle batches until `need` more bytes fit in the budget.
void evict_idle(bfs_server *s, size_t need) {
  for (size_t k = 0; k < s->batches.size() && s->used + need > s->budget;) {
    Batch *b = s->batches[k].get();
    if (!b->active && !b->in_flight) {
      s->used -= b->bytes;
      free_batch(b);
      s->batches.erase(s->batches.begin() + (long)k);
    } else {
      ++k;
    }
  }
}

// True when a batch other than `b` is running or a request of another
// graph is waiting.
bool others_busy(const bfs_server *s, const Batch *b) {
  for (const auto &o : s->batches)
    if (o.get() != b && (o->active || o->in_flight)) return true;
  for (const auto &w : s->waiting)
    if (w.first != b->g && !w.second.empty()) return true;
  return !s->inbox.empty();
}

int issue(bfs_server *s, Batch *b) {
  DeviceGuard dg(b->g->device);
  const int lv = chunk_levels(b->g, others_busy(s, b));
  return b->g->rp64 ? issue_chunk<int64_t>(b, lv) : issue_chunk<int32_t>(b, lv);
}

void worker_loop(bfs_server *s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    while (!s->inbox.empty()) {
      Request *r = s->inbox.front();
      s->inbox.pop_front();
      s->waiting[r->g].push_back(r);
    }
    bool busy = false;
    // finished chunks: retire lanes, admit into freed lanes, continue or free
    for (size_t k = 0; k < s->batches.size();) {
      Batch *b = s->batches[k].get();
      if (b->in_flight) {
        const hipError_t q = hipEventQuery(b->ev);
        if (q == hipErrorNotReady) {
          busy = true;
          ++k;
          continue;
        }
        b->in_flight = false;
        if (q != hipSuccess) fail_batch(s, b, "batch failed on the device");
        else retire(s, b);
      }
      admit(s, b);
      if (b->active) {
        if (issue(s, b) != BFS_OK) fail_batch(s, b, bfs_last_error());
        busy = busy || b->in_flight;
      }
      ++k;  // an empty batch stays allocated for the next request of its graph
    }
    // graphs with waiting requests and no batch to take them: open batches
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
      bfs_graph *g = it->first;
      const size_t need = batch_bytes(g);
      if (it->second.empty()) {
        it = s->waiting.erase(it);
        continue;
      }
      if (has_room(s, g)) {  // an existing batch of g will take them at its next boundary
        ++it;
        continue;
      }
      if (s->used + need > s->budget) evict_idle(s, need);
      if (s->used + need > s->budget) {
        ++it;
        continue;  // waits for memory
      }
      auto nb = std::make_unique<Batch>();
      if (!make_batch(nb.get(), g)) {
        free_batch(nb.get());
        ++it;
        continue;
      }
      s->used += need;
      Batch *b = nb.get();
      s->batches.push_back(std::move(nb));
      admit(s, b);  // may erase `it`'s entry
      it = s->waiting.lower_bound(g);
      if (issue(s, b) != BFS_OK) fail_batch(s, b, bfs_last_error());
      busy = true;
    }
    bool running = false;
    for (const auto &b : s->batches) running = running || b->active || b->in_flight;
    const bool idle = !running && s->waiting.empty() && s->inbox.empty();
    if (s->stop && idle) break;
    if (busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (!idle) {
      // requests wait for memory held by nothing in flight: cannot happen
      // unless the budget is below one batch (rejected at submit)
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(100));
      lk.lock();
    } else {
      s->cv.wait(lk, [s] { return s->stop || !s->inbox.empty(); });
    }
  }
}

}  // namespace

extern "C" {

int bfs_serve_create(size_t hbm_budget_bytes, int32_t max_lanes, bfs_server_t *out) {
  clear_error();
  if (!out) return fail(BFS_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (max_lanes < 1 || max_lanes > kLanes) return fail(BFS_ERR_INVALID_ARG, "max_lanes outside [1, 64]");
  if (hbm_budget_bytes == 0) return fail(BFS_ERR_INVALID_ARG, "zero budget");
  bfs_server *s = new (std::nothrow) bfs_server;
  if (!s) return fail(BFS_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->budget = hbm_budget_bytes;
  s->max_lanes = max_lanes;
  try {
    s->worker = std::thread(worker_loop, s);
  } catch (...) {
    delete s;
    return fail(BFS_ERR_OUT_OF_MEMORY, "cannot start the server thread");
  }
  *out = s;
  return BFS_OK;
}

int bfs_serve_destroy(bfs_server_t s) {
  clear_error();
  if (!s) return fail(BFS_ERR_INVALID_ARG, "null server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &b : s->batches) free_batch(b.get());
  delete s;
  return BFS_OK;
}

int bfs_serve_submit(bfs_server_t s, bfs_graph_t g, int32_t source, int32_t *dist_out,
                     int32_t *parent_out, uint64_t *ticket) {
  clear_error();
  if (!s || !g || !dist_out || !ticket) return fail(BFS_ERR_INVALID_ARG, "null argument");
  if (source < 0 || source >= g->n)
    return fail(BFS_ERR_INVALID_ARG, "source %d outside [0, %lld)", source, (long long)g->n);
  if (batch_bytes(g) > s->budget)
    return fail(BFS_ERR_OUT_OF_MEMORY, "a batch of this graph needs %zu bytes, budget is %zu",
                batch_bytes(g), s->budget);
  auto r = std::make_unique<Request>();
  r->g = g;
  r->source = source;
  r->dist = dist_out;
  r->parent = parent_out;
  r->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(BFS_ERR_INVALID_ARG, "server is stopping");
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    g->server_refs.fetch_add(1);
    s->inbox.push_back(r.get());
    s->reqs.emplace(r->ticket, std::move(r));
  }
  s->cv.notify_all();
  return BFS_OK;
}

int bfs_serve_poll(bfs_server_t s, uint64_t ticket, int32_t *state, bfs_req_stats *st) {
  clear_error();
  if (!s || !state) return fail(BFS_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BFS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  const Request *r = it->second.get();
  *state = r->state;
  if (st) {
    st->t_submit_ns = r->t_submit;
    st->t_admit_ns = r->t_admit;
    st->t_done_ns = r->t_done;
    st->levels = r->levels;
    st->batch_lanes = r->lanes_at_admit;
  }
  return BFS_OK;
}

}  // extern "C"
