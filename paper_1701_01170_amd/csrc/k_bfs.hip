// Breadth-first search steps (Sec. 6.1): push advance fused with the
// visited-bitmap filter, and pull advance over the unvisited frontier
// (Sec. 5.1 push vs. pull, Alg. 2).
//
// Visited state lives in two bitmaps, `old` and `live`.  At the start of level
// d: old = vertices at depth <= d, live = vertices at depth <= d - 1.
//  * push: every frontier vertex is marked in live; an edge (u, v) with v in
//    old is culled; otherwise v gets depth d + 1, u competes for parent[v] by
//    an unsigned atomic min (the smallest-id parent wins, -1 = 0xffffffff
//    loses to any id), and the first thread to set v's live bit appends v to
//    the next frontier exactly once.  Afterwards live = depth <= d + 1.
//  * pull: a vertex u is in the frontier iff it is in old and not in live.
//    Each unvisited v scans its ascending adjacency and stops at the first
//    frontier neighbour, which is therefore the smallest-id parent.  New
//    vertices are marked in live; the host then ORs old into live.
// The host swaps the two bitmaps after every level.
#include "k_advance.h"

namespace gr {

namespace {

struct BfsVisit {
  const uint32_t* __restrict__ old_bm;
  uint32_t* __restrict__ live_bm;
  int32_t* __restrict__ depth;
  int32_t* __restrict__ parent;
  int32_t next_depth;

  __device__ __forceinline__ int32_t seg_payload(int32_t) const { return 0; }
  __device__ __forceinline__ void on_frontier(int32_t u) const {
    atomicOr(&live_bm[u >> 5], 1u << (u & 31));
  }
  __device__ __forceinline__ bool visit(int32_t u, int32_t, int32_t v, int64_t) const {
    const uint32_t bit = 1u << (v & 31);
    const int32_t w = v >> 5;
    if (old_bm[w] & bit) return false;
    if (parent) atomicMin(reinterpret_cast<uint32_t*>(&parent[v]), (uint32_t)u);
    if (live_bm[w] & bit) return false;
    const uint32_t prev = atomicOr(&live_bm[w], bit);
    if (prev & bit) return false;
    depth[v] = next_depth;
    return true;
  }
};

__device__ __forceinline__ bool in_frontier(const uint32_t* old_bm, const uint32_t* live_bm,
                                            int32_t u) {
  const int32_t w = u >> 5;
  return ((old_bm[w] & ~live_bm[w]) >> (u & 31)) & 1u;
}

__device__ __forceinline__ void pull_emit(bool valid, int32_t v, int32_t found,
                                          uint32_t* live_bm, int32_t* depth, int32_t* parent,
                                          int32_t next_depth, int32_t* out_a, uint32_t* cnt_a,
                                          int32_t* out_u, uint32_t* cnt_u) {
  const bool hit = valid && found >= 0;
  const bool miss = valid && found < 0;
  if (hit) {
    depth[v] = next_depth;
    if (parent) parent[v] = found;
    atomicOr(&live_bm[v >> 5], 1u << (v & 31));
  }
  const uint32_t sa = wave_append(cnt_a, hit);
  if (hit) out_a[sa] = v;
  const uint32_t su = wave_append(cnt_u, miss);
  if (miss) out_u[su] = v;
}

// Pull with dynamic grouping: one lane per unvisited vertex for short lists
// (sequential ascending scan with early exit), one wavefront per vertex for
// lists longer than kPullLane (64 neighbours per step, first hit by ballot).
constexpr int kPullLane = 32;

__global__ __launch_bounds__(256) void k_bfs_pull_twc(
    const int32_t* __restrict__ unv, int32_t n_u, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, const uint32_t* __restrict__ old_bm,
    uint32_t* __restrict__ live_bm, int32_t* __restrict__ depth, int32_t* __restrict__ parent,
    int32_t next_depth, int32_t* __restrict__ out_a, uint32_t* __restrict__ cnt_a,
    int32_t* __restrict__ out_u, uint32_t* __restrict__ cnt_u, int64_t* __restrict__ inspected) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n_u;
  int32_t v = 0, rb = 0, re = 0;
  if (valid) {
    v = unv[i];
    rb = R[v];
    re = R[v + 1];
  }
  int32_t found = -1;
  int64_t scanned = 0;
  if (valid && re - rb <= kPullLane) {
    for (int32_t j = rb; j < re; ++j) {
      const int32_t u = C[j];
      ++scanned;
      if (in_frontier(old_bm, live_bm, u)) {
        found = u;
        break;
      }
    }
  }
  uint64_t big = __ballot(valid && re - rb > kPullLane);
  while (big) {
    const int l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const int32_t vb = __shfl(rb, l), ve = __shfl(re, l);
    int32_t f = -1;
    int64_t sc = 0;
    for (int32_t base = vb; base < ve; base += kWave) {
      const int32_t j = base + lane();
      int32_t u = -1;
      bool hit = false;
      if (j < ve) {
        u = C[j];
        hit = in_frontier(old_bm, live_bm, u);
      }
      const uint64_t b = __ballot(hit);
      sc += (ve - base) < kWave ? (ve - base) : kWave;
      if (b) {
        f = __shfl(u, __ffsll((unsigned long long)b) - 1);
        break;
      }
    }
    if (lane() == l) {
      found = f;
      scanned = sc;
    }
  }
  pull_emit(valid, v, found, live_bm, depth, parent, next_depth, out_a, cnt_a, out_u, cnt_u);
  if (inspected) {
    const int64_t s = wave_sum(scanned);
    if (lane() == 0 && s) atomicAdd((unsigned long long*)inspected, (unsigned long long)s);
  }
}

// Pull with fixed-width edge groups: GW lanes per unvisited vertex, every
// group checks GW consecutive neighbours per step; the lowest hit lane of the
// first step with a hit holds the smallest-id frontier neighbour.
template <int GW>
__global__ __launch_bounds__(256) void k_bfs_pull_groups(
    const int32_t* __restrict__ unv, int32_t n_u, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, const uint32_t* __restrict__ old_bm,
    uint32_t* __restrict__ live_bm, int32_t* __restrict__ depth, int32_t* __restrict__ parent,
    int32_t next_depth, int32_t* __restrict__ out_a, uint32_t* __restrict__ cnt_a,
    int32_t* __restrict__ out_u, uint32_t* __restrict__ cnt_u, int64_t* __restrict__ inspected) {
  static_assert(GW > 0 && GW < kWave && (kWave % GW) == 0, "group width");
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GW;
  const int sub = lane() % GW;
  const int gbase = lane() - sub;
  const bool valid = g < n_u;
  int32_t v = 0, rb = 0, re = 0;
  if (valid) {
    v = unv[g];
    rb = R[v];
    re = R[v + 1];
  }
  int32_t found = -1;
  int64_t scanned = 0;
  for (int32_t base = rb;; base += GW) {
    const bool active = valid && found < 0 && base < re;
    if (!__any(active)) break;
    const int32_t j = base + sub;
    int32_t u = -1;
    bool hit = false;
    if (active && j < re) {
      u = C[j];
      hit = in_frontier(old_bm, live_bm, u);
    }
    const uint64_t b = __ballot(hit);
    const uint64_t gm = (b >> gbase) & ((1ull << GW) - 1ull);
    const int src = gm ? gbase + __ffsll((unsigned long long)gm) - 1 : lane();
    const int32_t cand = __shfl(u, src);
    if (active) {
      scanned += (re - base) < GW ? (re - base) : GW;
      if (gm) found = cand;
    }
  }
  const bool leader = sub == 0;
  pull_emit(valid && leader, v, found, live_bm, depth, parent, next_depth, out_a, cnt_a, out_u,
            cnt_u);
  if (inspected) {
    const int64_t s = wave_sum(leader ? scanned : (int64_t)0);
    if (lane() == 0 && s) atomicAdd((unsigned long long*)inspected, (unsigned long long)s);
  }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_bfs_push_lb(const int32_t* frontier, const int32_t* offsets, int64_t n_f,
                              int64_t m_f, const int32_t* R, const int32_t* C,
                              const uint32_t* bm_old, uint32_t* bm_live, int32_t* depth,
                              int32_t* parent, int32_t next_depth, int32_t* out_q,
                              uint32_t* out_count, int chunk, hipStream_t st) {
  if (m_f <= 0) return hipSuccess;
  BfsVisit f{bm_old, bm_live, depth, parent, next_depth};
  k_push_lb<BfsVisit><<<blocks_for(m_f, chunk), kAdvBlock, 0, st>>>(
      frontier, offsets, (int32_t)n_f, (int32_t)m_f, R, C, f, out_q, out_count, chunk);
  return hipGetLastError();
}

hipError_t launch_bfs_push_light(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                 const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                                 int32_t* depth, int32_t* parent, int32_t next_depth,
                                 int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  if (n_f <= 0) return hipSuccess;
  BfsVisit f{bm_old, bm_live, depth, parent, next_depth};
  k_push_light<BfsVisit><<<blocks_for(n_f, kAdvBlock), kAdvBlock, 0, st>>>(
      frontier, (int32_t)n_f, R, C, f, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_bfs_push_twc(const int32_t* frontier, int64_t n_f, const int32_t* R,
                               const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                               int32_t* depth, int32_t* parent, int32_t next_depth,
                               int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  if (n_f <= 0) return hipSuccess;
  BfsVisit f{bm_old, bm_live, depth, parent, next_depth};
  k_push_twc<BfsVisit><<<blocks_for(n_f, kAdvBlock), kAdvBlock, 0, st>>>(
      frontier, (int32_t)n_f, R, C, f, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_bfs_pull(bool lb, const int32_t* unvisited, int64_t n_u, const int32_t* R,
                           const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                           int32_t* depth, int32_t* parent, int32_t next_depth,
                           int32_t* out_active, uint32_t* out_active_count,
                           int32_t* out_unvisited, uint32_t* out_unvisited_count,
                           int64_t* inspected, hipStream_t st) {
  if (n_u <= 0) return hipSuccess;
  if (lb) {
    constexpr int GW = 8;
    k_bfs_pull_groups<GW><<<blocks_for(n_u * GW, 256), 256, 0, st>>>(
        unvisited, (int32_t)n_u, R, C, bm_old, bm_live, depth, parent, next_depth, out_active,
        out_active_count, out_unvisited, out_unvisited_count, inspected);
  } else {
    k_bfs_pull_twc<<<blocks_for(n_u, 256), 256, 0, st>>>(
        unvisited, (int32_t)n_u, R, C, bm_old, bm_live, depth, parent, next_depth, out_active,
        out_active_count, out_unvisited, out_unvisited_count, inspected);
  }
  return hipGetLastError();
}

}  // namespace gr
