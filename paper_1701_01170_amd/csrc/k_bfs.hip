// Breadth-first search steps (Sec. 6.1): push advance fused with the
// visited-bitmap filter, and pull advance over the unvisited frontier
// (Sec. 5.1 push vs. pull, Alg. 2).
//
// Visited state is one array of 32-bit word pairs: at level d with parity p,
// word 2w + p ("old") holds vertices at depth <= d and word 2w + 1 - p ("live")
// holds vertices at depth <= d - 1 plus the vertices found so far at d + 1.
// One 8-byte load answers both questions for a vertex: a vertex u is in the
// current frontier iff it is in old and not in live.  During the level only
// vertices outside old get live bits, so that test stays valid for the whole
// level.  After the level the host ORs old into live (live = depth <= d + 1)
// and flips the parity.
//  * push: an edge (u, v) with v in old or live is culled; the first thread to
//    set v's live bit writes depth d + 1 and appends v to the next frontier
//    exactly once.  Parents: either every frontier in-neighbour competes with
//    an unsigned atomic min (-1 = 0xffffffff loses to any id), or, on
//    symmetric graphs, a fix-up pass scans each new vertex's ascending
//    adjacency for its first frontier neighbour (= the smallest-id parent).
//  * pull: each unvisited v scans its ascending adjacency and stops at the
//    first frontier neighbour, which is therefore the smallest-id parent.
#include "k_advance.h"
#include "k_dloop.h"

namespace gr {

namespace {

__device__ __forceinline__ uint2 bm_pair(const uint32_t* bm, int32_t w) {
  return reinterpret_cast<const uint2*>(bm)[w];
}

__device__ __forceinline__ int32_t caller_id(const int32_t* perm, int32_t v) {
  return perm ? perm[v] : v;
}

template <bool ATOMIC_PARENT>
struct BfsVisit {
  uint32_t* __restrict__ bm;
  int32_t* __restrict__ depth;
  int32_t* __restrict__ parent;
  const int32_t* __restrict__ perm;  // renumbered -> caller ids (nullable)
  int32_t next_depth;
  int32_t p;  // parity: old word = 2w + p

  using pay_t = int32_t;  // the frontier vertex's caller id (parents compare caller ids)
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return ATOMIC_PARENT && parent ? caller_id(perm, u) : 0;
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ bool probe(int32_t, int32_t, int32_t v, uint32_t) const {
    const uint2 x = bm_pair(bm, v >> 5);
    const uint32_t old = p ? x.y : x.x, live = p ? x.x : x.y;
    const uint32_t bit = 1u << (v & 31);
    if (ATOMIC_PARENT) return !(old & bit);
    return !((old | live) & bit);
  }
  __device__ __forceinline__ bool commit(int32_t, int32_t pu, int32_t v, uint32_t) const {
    const uint32_t bit = 1u << (v & 31);
    uint32_t* live = &bm[2 * (v >> 5) + 1 - p];
    if (ATOMIC_PARENT) {
      if (parent) atomicMin(reinterpret_cast<uint32_t*>(&parent[v]), (uint32_t)pu);
      if (*live & bit) return false;
    }
    const uint32_t prev = atomicOr(live, bit);
    if (prev & bit) return false;
    depth[v] = next_depth;
    return true;
  }
  // commit() for a lane's B edges in phases: parent minima (no return value
  // needed), then the live-word reads, then the OR of every still-clear bit,
  // so no edge waits for another edge's atomic.
  template <int B>
  __device__ __forceinline__ void commit_batch(const int32_t (&)[B], const int32_t (&pu)[B],
                                               const int32_t (&v)[B], const uint32_t (&)[B],
                                               const bool (&ok)[B], int (&code)[B]) const {
    uint32_t* live[B];
    uint32_t bit[B], w[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      bit[r] = 1u << (v[r] & 31);
      live[r] = &bm[2 * (v[r] >> 5) + 1 - p];
    }
    if (ATOMIC_PARENT && parent) {
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (ok[r]) atomicMin(reinterpret_cast<uint32_t*>(&parent[v[r]]), (uint32_t)pu[r]);
    }
#pragma unroll
    for (int r = 0; r < B; ++r) w[r] = (ATOMIC_PARENT && ok[r]) ? *live[r] : 0u;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const bool go = ok[r] && !(w[r] & bit[r]);
      w[r] = go ? atomicOr(live[r], bit[r]) : bit[r];
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      code[r] = (w[r] & bit[r]) ? 0 : 1;
      if (code[r]) depth[v[r]] = next_depth;
    }
  }
  // Device-predicated steps have no merge pass: each frontier vertex joins
  // live during its own level instead.  Push probes only test old, and
  // frontier vertices are in old, so this changes no decision of the level;
  // at its end live = depth <= d + 1, exactly what the merge would give.
  __device__ __forceinline__ void frontier_vertex(int32_t u) const {
    atomicOr(&bm[2 * (u >> 5) + 1 - p], 1u << (u & 31));
  }
  __device__ __forceinline__ BfsVisit prepare(const Ctrl*, int) const { return *this; }
  __device__ __forceinline__ void advance(Ctrl*, int, bool) const {}
};

// Push without returning atomics (for levels that discover many vertices):
// every edge into a vertex outside old and live stores a one-byte mark; all
// writers store the same value, so the race is benign.  k_bfs_mark_compact
// then turns the marks into depths, live bits and an ordered next frontier.
// With parent (nullable) every such edge also takes the atomic minimum of the
// parent, whose result nobody waits for (canonical parents without the
// fix-up scan; live holds no vertex of this level, so the probe passes every
// edge into a vertex not in old).
struct BfsMark {
  const uint32_t* __restrict__ bm;
  uint8_t* __restrict__ marks;
  int32_t p;
  int32_t* __restrict__ parent;
  const int32_t* __restrict__ perm;

  using pay_t = int32_t;  // the frontier vertex's caller id when parents are taken
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = false;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return parent ? caller_id(perm, u) : 0;
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ bool probe(int32_t, int32_t, int32_t v, uint32_t) const {
    const uint2 x = bm_pair(bm, v >> 5);
    return !(((x.x | x.y) >> (v & 31)) & 1u);
  }
  __device__ __forceinline__ bool commit(int32_t, int32_t pu, int32_t v, uint32_t) const {
    if (parent) {
      // frontier rows are handled roughly in ascending order, so most edges
      // find a smaller parent already and skip the atomic
      uint32_t* pv = reinterpret_cast<uint32_t*>(&parent[v]);
      if ((uint32_t)pu < *pv) atomicMin(pv, (uint32_t)pu);
    }
    marks[v] = 1;
    return false;
  }
};

// Idempotent push (Sec. 5.2, idempotent vs. non-idempotent operations).  The
// BFS visit is idempotent -- every discoverer of v stores the same depth -- so
// this advance takes no atomic at all.  Repeated discoveries of a vertex are
// culled by inexpensive, inexact heuristics (the paper's global bitmask, block
// level history table and warp level table), in this order:
//   probe   the visited bitmap (old: depth <= d; one bit, cache resident);
//   HISTORY a per-workgroup table in LDS, slot = multiplicative hash of v: v
//           is dropped when its slot holds v;
//   WAVE    a per-wavefront table of 128 slots: the lanes of one batch write
//           their v, then those that read their own v back write a tag (lane,
//           edge); of the lanes holding the same v only the one whose tag
//           survives keeps it;
//   LABEL   the depth label: v is dropped when some lane already wrote d + 1.
// A survivor stores depth d + 1, enters the history table and is appended to
// the candidate list.  Each heuristic drops v only when some lane keeps v (a
// table slot holds v only if a lane kept it; a written label was written by a
// lane that keeps v), so no vertex is lost; races between wavefronts only let
// duplicates through.  k_bfs_idem_filter removes those exactly.
constexpr int kIdemWaveSlots = 128;

template <int LOG_H>
__device__ __forceinline__ int32_t* idem_history() {
  __shared__ int32_t t[1 << LOG_H];
  return t;
}

__device__ __forceinline__ int32_t* idem_wave_table(int which) {
  __shared__ int32_t t[2][512 / kWave][kIdemWaveSlots];  // up to 512-thread workgroups
  return t[which][threadIdx.x / kWave];
}

template <int LOG_H>
struct BfsIdem {
  const uint32_t* __restrict__ bm;
  int32_t* __restrict__ depth;
  int32_t next_depth;
  int32_t p;
  uint32_t culls;    // GR_IDEM_CULL_* bits that are on
  uint32_t out_cap;  // candidate list capacity

  using pay_t = int32_t;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t) const { return 0; }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ static uint32_t slot(int32_t v) {
    return ((uint32_t)v * 2654435761u) >> (32 - LOG_H);
  }
  __device__ __forceinline__ void block_init() const {
    int32_t* h = idem_history<LOG_H>();
    for (int i = threadIdx.x; i < (1 << LOG_H); i += (int)blockDim.x) h[i] = -1;
  }
  __device__ __forceinline__ bool probe(int32_t, int32_t, int32_t v, uint32_t) const {
    const uint2 x = bm_pair(bm, v >> 5);
    return !(((p ? x.y : x.x) >> (v & 31)) & 1u);
  }
  __device__ __forceinline__ bool commit(int32_t, int32_t, int32_t, uint32_t) const { return false; }
  template <int B>
  __device__ __forceinline__ void commit_batch(const int32_t (&)[B], const int32_t (&)[B],
                                               const int32_t (&v)[B], const uint32_t (&)[B],
                                               const bool (&ok)[B], int (&code)[B]) const {
    int32_t* hist = idem_history<LOG_H>();
    bool keep[B];
#pragma unroll
    for (int r = 0; r < B; ++r) keep[r] = ok[r];
    if (culls & GR_IDEM_CULL_HISTORY) {
#pragma unroll
      for (int r = 0; r < B; ++r) keep[r] = keep[r] && hist[slot(v[r])] != v[r];
    }
    if (culls & GR_IDEM_CULL_WAVE) {
      // every lane of the wavefront is here (edge_batch's contract)
      int32_t* vals = idem_wave_table(0);
      int32_t* tags = idem_wave_table(1);
      bool mine[B];
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (keep[r]) vals[v[r] & (kIdemWaveSlots - 1)] = v[r];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int r = 0; r < B; ++r) mine[r] = keep[r] && vals[v[r] & (kIdemWaveSlots - 1)] == v[r];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (mine[r]) tags[v[r] & (kIdemWaveSlots - 1)] = lane() * B + r;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (mine[r]) keep[r] = tags[v[r] & (kIdemWaveSlots - 1)] == lane() * B + r;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    if (culls & GR_IDEM_CULL_LABEL) {
      int32_t dv[B];
#pragma unroll
      for (int r = 0; r < B; ++r) dv[r] = keep[r] ? depth[v[r]] : -1;
#pragma unroll
      for (int r = 0; r < B; ++r) keep[r] = keep[r] && dv[r] < 0;
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      code[r] = keep[r] ? 1 : 0;
      if (keep[r]) {
        depth[v[r]] = next_depth;
        if (culls & GR_IDEM_CULL_HISTORY) hist[slot(v[r])] = v[r];
      }
    }
  }
};

// The exact filter after the idempotent advance.  Each candidate's live bit is
// set with an atomic OR and the lane that set it appends the vertex, so the
// next frontier holds every new vertex once.  When the candidates outgrew the
// list (more than cap), the list is incomplete and the pass instead reads the
// depth labels of all V vertices: every vertex discovered this level has depth
// d + 1 (its keeper wrote it) and no live bit yet.  Grid-stride; the branch is
// the same for every workgroup.
__global__ __launch_bounds__(256) void k_bfs_idem_filter(const int32_t* __restrict__ cand,
                                                         const uint32_t* __restrict__ n_cand,
                                                         int64_t cap, int64_t V,
                                                         uint32_t* __restrict__ bm, int p,
                                                         const int32_t* __restrict__ depth,
                                                         int32_t next_depth,
                                                         int32_t* __restrict__ out_q,
                                                         uint32_t* __restrict__ out_count) {
  const int64_t n = *n_cand;
  const int64_t stride = (int64_t)gridDim.x * 256;
  if (n <= cap) {
    for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < n; b0 += stride) {
      const int64_t i = b0 + threadIdx.x;
      bool first = false;
      int32_t v = 0;
      if (i < n) {
        v = cand[i];
        const uint32_t bit = 1u << (v & 31);
        first = !(atomicOr(&bm[2 * (v >> 5) + 1 - p], bit) & bit);
      }
      const uint32_t a = block_append<256>(first ? 1u : 0u, out_count);
      if (first) out_q[a] = v;
    }
  } else {
    const int64_t nw = (V + 31) / 32;
    for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < nw; b0 += stride) {
      const int64_t w = b0 + threadIdx.x;
      uint32_t mask = 0;
      if (w < nw) {
        const int64_t v0 = w * 32;
        for (int b = 0; b < 32; ++b)
          if (v0 + b < V && depth[v0 + b] == next_depth) mask |= 1u << b;
        // this thread is the only writer of the word in this branch
        if (mask) bm[2 * w + 1 - p] |= mask;
      }
      append_mask<256>(mask, w, out_q, out_count);
    }
  }
}

// One thread per bitmap word (32 vertices): gather the marks, clear them, set
// the live bits (the thread owns the word), write depths and append the new
// vertices in ascending order within each workgroup (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_bfs_mark_compact(uint8_t* __restrict__ marks, int64_t V,
                                                          uint32_t* __restrict__ bm, int p,
                                                          int32_t* __restrict__ depth,
                                                          int32_t next_depth,
                                                          int32_t* __restrict__ out_q,
                                                          uint32_t* __restrict__ out_count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t mask = take_marks(marks, w, V);
  if (mask) bm[2 * w + 1 - p] |= mask;
  uint32_t base = block_append<256>(__popc(mask), out_count);
  while (mask) {
    const int b = __ffs(mask) - 1;
    mask &= mask - 1;
    const int32_t v = (int32_t)(w * 32 + b);
    depth[v] = next_depth;
    out_q[base++] = v;
  }
}

__device__ __forceinline__ bool in_frontier(const uint32_t* bm, int p, int32_t u) {
  const uint2 x = bm_pair(bm, u >> 5);
  const uint32_t f = p ? (x.y & ~x.x) : (x.x & ~x.y);
  return (f >> (u & 31)) & 1u;
}

// Smallest-id frontier neighbour of the vertex owned by each lane, with
// dynamic grouping: a lane scans a list of at most LANE_MAX neighbours by
// itself (ascending, early exit); longer lists are scanned by the whole
// wavefront, U * 64 neighbours per step with U independent loads per lane,
// the first hit taken by ballot.  Returns -1 when there is none; *scanned
// counts neighbours read.
template <int LANE_MAX>
__device__ __forceinline__ int32_t first_frontier_nbr(bool valid, int32_t rb, int32_t re,
                                                      const int32_t* __restrict__ C,
                                                      const uint32_t* __restrict__ bm, int p,
                                                      int64_t* scanned) {
  constexpr int U = 8;
  int32_t found = -1;
  int64_t sc = 0;
  if (valid && re - rb <= LANE_MAX) {
    // U neighbours per step: U independent loads, then U independent probes
    for (int32_t j0 = rb; j0 < re && found < 0; j0 += U) {
      int32_t u[U];
      bool hit[U];
#pragma unroll
      for (int r = 0; r < U; ++r) u[r] = j0 + r < re ? C[j0 + r] : -1;
#pragma unroll
      for (int r = 0; r < U; ++r) hit[r] = u[r] >= 0 && in_frontier(bm, p, u[r]);
#pragma unroll
      for (int r = U - 1; r >= 0; --r)
        if (hit[r]) found = u[r];
      sc += (re - j0) < U ? (re - j0) : U;
    }
  }
  uint64_t big = __ballot(valid && re - rb > LANE_MAX);
  while (big) {
    const int l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const int32_t vb = __shfl(rb, l), ve = __shfl(re, l);
    int32_t f = -1;
    int64_t s2 = 0;
    for (int32_t base = vb; base < ve; base += U * kWave) {
      int32_t u[U];
      bool hit[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int32_t j = base + r * kWave + lane();
        u[r] = j < ve ? C[j] : -1;
      }
#pragma unroll
      for (int r = 0; r < U; ++r) hit[r] = u[r] >= 0 && in_frontier(bm, p, u[r]);
      bool done = false;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const uint64_t b = __ballot(hit[r]);
        if (!done && b) {
          f = __shfl(u[r], __ffsll((unsigned long long)b) - 1);
          s2 += (int64_t)r * kWave + __ffsll((unsigned long long)b);
          done = true;
        }
      }
      if (done) break;
      s2 += (ve - base) < U * kWave ? (ve - base) : U * kWave;
    }
    if (lane() == l) {
      found = f;
      sc = s2;
    }
  }
  *scanned = sc;
  return found;
}

// Pull over the visited bitmap (Alg. 2, with the unvisited set read from the
// bitmap instead of a generated list): each wavefront owns kPullRuns runs of
// 64 consecutive vertices, i.e. their bitmap words, which no other wavefront
// writes during the step.  The runs of a wavefront are spread over the whole
// id range (run k of wavefront w of workgroup b is run (k G + b) NW + w), so
// that every workgroup gets a similar share of unvisited vertices even when
// the ids are degree ordered (hubs, reached first, at the low ids).  A vertex outside old scans its ascending
// adjacency for its first frontier neighbour (the smallest-id parent); the
// wavefront ORs its hits into live with one plain store per word and the
// workgroup appends them to the next frontier with a single atomic.
// GW = 1: one lane per vertex (dynamic grouping: lists longer than 32 go to
// the whole wavefront); GW > 1: GW lanes per vertex, GW neighbours per step
// (lists longer than 64 go to the whole wavefront).
// The step is a chain of dependent loads (row bounds, neighbour, frontier
// bit), so resident waves hide its latency: the kernel asks for 8 waves per
// SIMD (its scalar registers alone would allow 7; the few that spill go to
// vector-register lanes, not memory).
constexpr int kPullRuns = 8;
constexpr int kPullBatch = 4;  // runs whose first neighbours are probed together
static_assert(kPullRuns % kPullBatch == 0, "whole batches");

template <int GW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_bfs_pull_bm(
    int64_t V, const int32_t* __restrict__ R, const int32_t* __restrict__ C,
    uint32_t* __restrict__ bm, int p, int32_t* __restrict__ depth, int32_t* __restrict__ parent,
    const int32_t* __restrict__ perm, int32_t next_depth, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count, int64_t* __restrict__ inspected,
    int32_t* __restrict__ rem_q, uint32_t* __restrict__ rem_count) {
  static_assert(GW >= 1 && GW < kWave && (kWave % GW) == 0, "group width");
  constexpr int NW = 256 / kWave;
  constexpr int VPR = kWave / GW;  // vertices per sub-round
  __shared__ uint32_t s_cnt[NW];
  __shared__ int64_t s_insp[NW];
  __shared__ uint32_t s_base;
  const int w = threadIdx.x / kWave;
  // first vertex of run k of this wavefront
  auto run_v0 = [&](int k) -> int64_t {
    return (((int64_t)k * gridDim.x + blockIdx.x) * NW + w) * kWave;
  };
  uint32_t hits = 0;  // bit k: vertex run_v0(k) + lane was found
  uint32_t rems = 0;  // bit k: that vertex has neighbours and stays unvisited
  int64_t scanned = 0;
  // GW == 1: the smallest-id neighbour of every candidate of kPullBatch runs
  // is probed up front, the loads of those runs in flight together (three
  // dependent rounds per batch instead of three per run).  On a wide pull
  // level most unvisited vertices find their parent there (a low-id hub in
  // the frontier); the per-run scan below continues only the others.
  int32_t prb[kPullBatch], pre[kPullBatch], pu[kPullBatch];
  bool pc[kPullBatch], ph[kPullBatch];
#pragma unroll
  for (int k = 0; k < kPullRuns; ++k) {
    const int64_t v0 = run_v0(k);
    if (v0 >= V) break;  // uniform across the wavefront; run_v0 grows with k
    const int kb = k % kPullBatch;
    if constexpr (GW == 1) {
      if (kb == 0) {
#pragma unroll
        for (int j = 0; j < kPullBatch; ++j) {
          const int64_t v = run_v0(k + j) + lane();
          pc[j] = false;
          prb[j] = pre[j] = 0;
          if (v < V) {
            const uint2 x = bm_pair(bm, (int32_t)(v >> 5));
            if (!(((p ? x.y : x.x) >> (v & 31)) & 1u)) {
              prb[j] = R[v];
              pre[j] = R[v + 1];
              pc[j] = pre[j] > prb[j];
            }
          }
        }
#pragma unroll
        for (int j = 0; j < kPullBatch; ++j) pu[j] = pc[j] ? C[prb[j]] : 0;
#pragma unroll
        for (int j = 0; j < kPullBatch; ++j) ph[j] = pc[j] && in_frontier(bm, p, pu[j]);
      }
    }
    uint64_t hb = 0;
    if constexpr (GW == 1) {
      const int64_t v = v0 + lane();
      const bool cand = pc[kb], first = cand && ph[kb];
      int64_t sc = 0;
      const int32_t rest = first_frontier_nbr<32>(cand && !first, prb[kb] + 1, pre[kb], C, bm, p,
                                                  &sc);
      const int32_t found = first ? pu[kb] : rest;
      if (cand) sc += 1;
      const bool hit = cand && found >= 0;
      if (cand && !hit) rems |= 1u << k;
      if (hit) {
        depth[v] = next_depth;
        if (parent) parent[v] = caller_id(perm, found);
      }
      hb = __ballot(hit);
      scanned += sc;
    } else {
      const int g = lane() / GW, sub = lane() % GW, gbase = g * GW;
      const bool leader = sub == 0;
      uint64_t rb_all = 0;  // the run's vertices that stay unvisited with neighbours
      for (int s = 0; s < GW; ++s) {
        const int64_t v = v0 + s * VPR + g;
        bool cand = false;
        int32_t rb = 0, re = 0;
        if (v < V) {
          const uint2 x = bm_pair(bm, (int32_t)(v >> 5));
          if (!(((p ? x.y : x.x) >> (v & 31)) & 1u)) {
            rb = R[v];
            re = R[v + 1];
            cand = re > rb;
          }
        }
        const bool small = cand && re - rb <= kWave;
        int32_t found = -1;
        int64_t sc = 0;
        for (int32_t b = rb;; b += GW) {
          const bool active = small && found < 0 && b < re;
          if (!__any(active)) break;
          const int32_t j = b + sub;
          int32_t u = -1;
          bool h = false;
          if (active && j < re) {
            u = C[j];
            h = in_frontier(bm, p, u);
          }
          const uint64_t bb = __ballot(h);
          const uint64_t gm = (bb >> gbase) & ((1ull << GW) - 1ull);
          const int src = gm ? gbase + __ffsll((unsigned long long)gm) - 1 : lane();
          const int32_t cnd = __shfl(u, src);
          if (active) {
            sc += (re - b) < GW ? (re - b) : GW;
            if (gm) found = cnd;
          }
        }
        int64_t scb = 0;
        const bool big = leader && cand && !small;
        const int32_t fb = first_frontier_nbr<0>(big, rb, re, C, bm, p, &scb);
        if (big) {
          found = fb;
          sc = scb;
        }
        const bool hit = leader && cand && found >= 0;
        if (hit) {
          depth[v] = next_depth;
          if (parent) parent[v] = caller_id(perm, found);
        }
        const uint64_t lb = __ballot(hit);  // bit g * GW for group g
        const uint64_t lr = __ballot(leader && cand && !hit);
        uint64_t m = 0, mr = 0;
        for (int q = 0; q < VPR; ++q) {
          m |= ((lb >> (q * GW)) & 1ull) << q;
          mr |= ((lr >> (q * GW)) & 1ull) << q;
        }
        hb |= m << (s * VPR);
        rb_all |= mr << (s * VPR);
        if (leader) scanned += sc;
      }
      if ((rb_all >> lane()) & 1ull) rems |= 1u << k;
    }
    // live bits of the run's two words (owned by this wavefront)
    const int64_t w0 = v0 >> 5;
    if (lane() == 0 && (uint32_t)hb) bm[2 * w0 + 1 - p] |= (uint32_t)hb;
    if (lane() == 32 && (uint32_t)(hb >> 32)) bm[2 * (w0 + 1) + 1 - p] |= (uint32_t)(hb >> 32);
    if ((hb >> lane()) & 1ull) hits |= 1u << k;
  }
  // one append (and one inspected-count update) per workgroup
  const uint32_t n = __popc(hits);
  const uint32_t inc = wave_incl_scan(n);
  const int64_t ws = wave_sum(scanned);
  if (lane() == kWave - 1) s_cnt[w] = inc;
  if (lane() == 0) s_insp[w] = ws;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    int64_t ins = 0;
    for (int i = 0; i < NW; ++i) {
      const uint32_t c = s_cnt[i];
      s_cnt[i] = tot;
      tot += c;
      ins += s_insp[i];
    }
    s_base = tot ? atomicAdd(out_count, tot) : 0u;
    if (inspected && ins) atomicAdd(reinterpret_cast<unsigned long long*>(inspected), (unsigned long long)ins);
  }
  __syncthreads();
  uint32_t slot = s_base + s_cnt[w] + inc - n;
  for (int k = 0; k < kPullRuns; ++k)
    if ((hits >> k) & 1u) out_q[slot++] = (int32_t)(run_v0(k) + lane());
  // the vertices still unvisited (and not isolated): the next pull level's list
  if (rem_q) {
    uint32_t rs = block_append<256>(__popc(rems), rem_count);
    for (int k = 0; k < kPullRuns; ++k)
      if ((rems >> k) & 1u) rem_q[rs++] = (int32_t)(run_v0(k) + lane());
  }
}

// Pull over a list of unvisited vertices (those the previous pull level left,
// all with neighbours): lane per vertex, the same smallest-id parent scan as
// the bitmap pull.  Bitmap words are shared by the lanes of different
// workgroups here, so live bits are set with an atomic OR.  Vertices that
// stay unvisited form the next list.
__global__ __launch_bounds__(256) void k_bfs_pull_list(
    const int32_t* __restrict__ list, const uint32_t* __restrict__ n_list,
    const int32_t* __restrict__ R, const int32_t* __restrict__ C, uint32_t* __restrict__ bm, int p,
    int32_t* __restrict__ depth, int32_t* __restrict__ parent, const int32_t* __restrict__ perm,
    int32_t next_depth, int32_t* __restrict__ out_q, uint32_t* __restrict__ out_count,
    int64_t* __restrict__ inspected, int32_t* __restrict__ rem_q,
    uint32_t* __restrict__ rem_count) {
  __shared__ int64_t s_insp[256 / kWave];
  const int64_t n = *n_list;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  int32_t v = 0, rb = 0, re = 0;
  bool cand = false;
  if (valid) {
    v = list[i];
    // a list entry reached since the list was made is dropped
    const uint2 x = bm_pair(bm, v >> 5);
    cand = !(((x.x | x.y) >> (v & 31)) & 1u);
    if (cand) {
      rb = R[v];
      re = R[v + 1];
    }
  }
  int64_t sc = 0;
  const int32_t found = first_frontier_nbr<32>(cand, rb, re, C, bm, p, &sc);
  const bool hit = cand && found >= 0;
  if (hit) {
    depth[v] = next_depth;
    if (parent) parent[v] = caller_id(perm, found);
    atomicOr(&bm[2 * (v >> 5) + 1 - p], 1u << (v & 31));
  }
  const uint32_t a = block_append<256>(hit ? 1u : 0u, out_count);
  if (hit) out_q[a] = v;
  const uint32_t b = block_append<256>(cand && !hit ? 1u : 0u, rem_count);
  if (cand && !hit) rem_q[b] = v;
  const int64_t ws = wave_sum(sc);
  if (lane() == 0) s_insp[threadIdx.x / kWave] = ws;
  __syncthreads();
  if (threadIdx.x == 0 && inspected) {
    int64_t t = 0;
    for (int k = 0; k < 256 / kWave; ++k) t += s_insp[k];
    if (t) atomicAdd(reinterpret_cast<unsigned long long*>(inspected), (unsigned long long)t);
  }
}

// Parents of the vertices a push step discovered (symmetric graphs): the
// first frontier neighbour in ascending order.
__global__ __launch_bounds__(256) void k_bfs_parent_fixup(const int32_t* __restrict__ list,
                                                          const uint32_t* __restrict__ count,
                                                          const int32_t* __restrict__ R,
                                                          const int32_t* __restrict__ C,
                                                          const uint32_t* __restrict__ bm, int p,
                                                          int32_t* __restrict__ parent,
                                                          const int32_t* __restrict__ perm) {
  const int64_t n = *count;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)blockIdx.x * blockDim.x >= n) return;  // whole block past the end
  const bool valid = i < n;
  int32_t v = 0, rb = 0, re = 0;
  if (valid) {
    v = list[i];
    rb = R[v];
    re = R[v + 1];
  }
  int64_t scanned;
  const int32_t par = first_frontier_nbr<32>(valid, rb, re, C, bm, p, &scanned);
  if (valid) parent[v] = caller_id(perm, par);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_bfs_push(int mode, bool atomic_parent, const int32_t* frontier,
                           const int32_t* offsets, const int32_t* rstart,
                           const int32_t* chunk_start, int64_t n_f, int64_t m_f, const int32_t* R,
                           const int32_t* C, uint32_t* bm, int p, int32_t* depth, int32_t* parent,
                           const int32_t* perm, int32_t next_depth, int32_t* out_q,
                           uint32_t* out_count, const AdvCfg& cfg, hipStream_t st) {
  if (atomic_parent) {
    BfsVisit<true> f{bm, depth, parent, perm, next_depth, p};
    return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, out_q,
                         out_count, cfg, st);
  }
  BfsVisit<false> f{bm, depth, nullptr, nullptr, next_depth, p};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, out_q,
                       out_count, cfg, st);
}

hipError_t launch_bfs_push_marks(int mode, const int32_t* frontier, const int32_t* offsets,
                                 const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                 int64_t m_f, const int32_t* R, const int32_t* C, uint32_t* bm,
                                 int p, uint8_t* marks, int32_t* parent, const int32_t* perm,
                                 const AdvCfg& cfg, hipStream_t st) {
  BfsMark f{bm, marks, p, parent, perm};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st);
}

hipError_t launch_bfs_push_idem(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C,
                                const uint32_t* bm, int p, int32_t* depth, int32_t next_depth,
                                uint32_t culls, int log_h, int32_t* cand, uint32_t* cand_count,
                                int64_t cap, const AdvCfg& cfg, hipStream_t st) {
  const uint32_t c32 = cap < (int64_t)UINT32_MAX ? (uint32_t)cap : UINT32_MAX;
  if (log_h == 8) {
    BfsIdem<8> f{bm, depth, next_depth, p, culls, c32};
    return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, cand,
                         cand_count, cfg, st);
  }
  if (log_h == 12) {
    BfsIdem<12> f{bm, depth, next_depth, p, culls, c32};
    return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, cand,
                         cand_count, cfg, st);
  }
  BfsIdem<10> f{bm, depth, next_depth, p, culls, c32};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, cand,
                       cand_count, cfg, st);
}

hipError_t launch_bfs_idem_filter(const int32_t* cand, const uint32_t* cand_count, int64_t cap,
                                  int64_t V, uint32_t* bm, int p, const int32_t* depth,
                                  int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                  hipStream_t st) {
  int64_t g = blocks_for(std::max<int64_t>(cap, (V + 31) / 32), 256);
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  k_bfs_idem_filter<<<(unsigned)g, 256, 0, st>>>(cand, cand_count, cap, V, bm, p, depth,
                                                 next_depth, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_bfs_mark_compact(uint8_t* marks, int64_t V, uint32_t* bm, int p, int32_t* depth,
                                   int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                   hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  k_bfs_mark_compact<<<blocks_for(n_words, 256), 256, 0, st>>>(marks, V, bm, p, depth, next_depth,
                                                               out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_bfs_parent_fixup(const int32_t* list, const uint32_t* count, int64_t max_count,
                                   const int32_t* R, const int32_t* C, const uint32_t* bm, int p,
                                   int32_t* parent, const int32_t* perm, hipStream_t st) {
  if (max_count <= 0) return hipSuccess;
  k_bfs_parent_fixup<<<blocks_for(max_count, 256), 256, 0, st>>>(list, count, R, C, bm, p, parent,
                                                                 perm);
  return hipGetLastError();
}

hipError_t launch_bfs_pull(bool lb, int64_t V, const int32_t* R, const int32_t* C, uint32_t* bm,
                           int p, int32_t* depth, int32_t* parent, const int32_t* perm,
                           int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                           int64_t* inspected, int32_t* rem_q, uint32_t* rem_count,
                           hipStream_t st) {
  if (V <= 0) return hipSuccess;
  const unsigned g = blocks_for(V, 256 * kPullRuns);
  if (lb)
    k_bfs_pull_bm<4><<<g, 256, 0, st>>>(V, R, C, bm, p, depth, parent, perm, next_depth, out_q,
                                        out_count, inspected, rem_q, rem_count);
  else
    k_bfs_pull_bm<1><<<g, 256, 0, st>>>(V, R, C, bm, p, depth, parent, perm, next_depth, out_q,
                                        out_count, inspected, rem_q, rem_count);
  return hipGetLastError();
}

hipError_t launch_bfs_pull_list(const int32_t* list, const uint32_t* n_list, int64_t max_n,
                                const int32_t* R, const int32_t* C, uint32_t* bm, int p,
                                int32_t* depth, int32_t* parent, const int32_t* perm,
                                int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                int64_t* inspected, int32_t* rem_q, uint32_t* rem_count,
                                hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  k_bfs_pull_list<<<blocks_for(max_n, 256), 256, 0, st>>>(list, n_list, R, C, bm, p, depth,
                                                          parent, perm, next_depth, out_q,
                                                          out_count, inspected, rem_q, rem_count);
  return hipGetLastError();
}

hipError_t launch_bfs_dstep(const DlArgs& a, uint32_t* bm, int p, int32_t* depth, int32_t* parent,
                            const int32_t* perm, int32_t next_depth, int n_blocks, hipStream_t st) {
  const BfsVisit<true> f{bm, depth, parent, perm, next_depth, p};
  k_dstep<BfsVisit<true>><<<n_blocks, kAdvBlock, 0, st>>>(a, f);
  return hipGetLastError();
}

}  // namespace gr
