// Single-source shortest paths (Sec. 6.2, Alg. 1): push advance whose fused
// functor relaxes every edge of the frontier with an atomic minimum
// (Update_Label), and a fused filter that lets each improved vertex into the
// next frontier once per iteration via an output-queue tag (Set_Pred /
// Remove_Redundant).
//
// Distance and predecessor are packed into one 64-bit key per vertex,
// key = dist << 32 | pred, so a single 64-bit atomic minimum keeps the
// lexicographically smallest (distance, predecessor) pair.  Every vertex
// relaxes its out-edges at least once with its final distance, hence the final
// key holds the true distance and the smallest-id predecessor among all tight
// in-edges.  Unreached vertices keep ~0 (distance UINT32_MAX, predecessor -1).
//
// Optional two-level priority queue (Sec. 5.1: the near / far split of the
// output frontier, a delta-stepping style binning): an improved vertex joins
// the next frontier only if its distance is below the threshold T; otherwise
// it goes to a far pile (at most once per far-pile generation).  When the
// frontier runs dry, T grows by delta and the far pile is split into the new
// frontier (T <= dist < T + delta), the next far pile (dist >= T + delta) and
// stale entries (dist < T: already expanded with that distance).  Every vertex
// is still expanded with its final distance, so results are unchanged.
#include "k_advance.h"
#include "k_dloop.h"

namespace gr {

namespace {

// Payload of a frontier vertex: its distance.  The predecessor written into
// a neighbour's key is the vertex's caller id (so ties between predecessors
// compare caller ids); the probe does not need it: it passes every edge that
// does not lengthen the distance, and the atomic minimum settles ties.
__device__ __forceinline__ uint32_t caller_id(const int32_t* perm, int32_t u) {
  return (uint32_t)(perm ? perm[u] : u);
}

struct SsspVisit {
  const uint32_t* __restrict__ W;
  unsigned long long* __restrict__ keys;
  int32_t* __restrict__ tags;
  const int32_t* __restrict__ perm;
  int32_t next_tag;

  using pay_t = int32_t;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return (int32_t)(uint32_t)(keys[u] >> 32);
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t e) const { return W[e]; }
  __device__ __forceinline__ bool probe(int32_t, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    if (cand >= 0xffffffffull) return false;  // cannot be a shortest distance (range checked at entry)
    return cand <= (keys[v] >> 32);            // keys only decrease: otherwise nothing to gain
  }
  __device__ __forceinline__ bool commit(int32_t u, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    const unsigned long long nk = (cand << 32) | caller_id(perm, u);
    const unsigned long long old = atomicMin(&keys[v], nk);
    if (cand >= (old >> 32)) return false;     // no distance improvement (at most a better pred)
    return atomicExch(&tags[v], next_tag) != next_tag;
  }
  // commit() for a lane's B edges in phases: all atomic minima, then the tag
  // exchanges of the improved vertices, so no edge waits for another's atomic.
  template <int B>
  __device__ __forceinline__ void commit_batch(const int32_t (&u)[B], const int32_t (&du)[B],
                                               const int32_t (&v)[B], const uint32_t (&w)[B],
                                               const bool (&ok)[B], int (&code)[B]) const {
    unsigned long long nk[B];
    int32_t prev[B];
#pragma unroll
    for (int r = 0; r < B; ++r)
      nk[r] = (((uint64_t)(uint32_t)du[r] + (uint64_t)w[r]) << 32) | (ok[r] ? caller_id(perm, u[r]) : 0u);
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const unsigned long long old = ok[r] ? atomicMin(&keys[v[r]], nk[r]) : 0ull;
      code[r] = ok[r] && (nk[r] >> 32) < (old >> 32);
    }
#pragma unroll
    for (int r = 0; r < B; ++r) prev[r] = code[r] ? atomicExch(&tags[v[r]], next_tag) : next_tag;
#pragma unroll
    for (int r = 0; r < B; ++r) code[r] = prev[r] != next_tag;
  }
  __device__ __forceinline__ void frontier_vertex(int32_t) const {}
  __device__ __forceinline__ SsspVisit prepare(const Ctrl*, int) const { return *this; }
  __device__ __forceinline__ void advance(Ctrl*, int, bool) const {}
};

// Relaxation without a returning atomic (for iterations with many frontier
// edges): each edge that lowers the key issues an atomic minimum whose result
// nobody waits for, and each edge that lowers the distance seen at its probe
// stores a one-byte mark (all writers store the same value).  A key only
// decreases, so a vertex gets a mark exactly when its distance decreased in
// this iteration, by this edge or by a concurrent one: the marks are the
// next frontier, which k_sssp_mark_compact lists in ascending order.
//
// With FILTER, a 16-bit distance mirror (min(dist, 0xffff) of an earlier
// moment, refreshed by the compaction for every marked vertex) screens the
// edges first.  Distances only decrease, so a mirror value below 0xffff is an
// upper bound of the current distance: an edge whose candidate exceeds it can
// neither shorten the distance nor tie it, and skips the 8-byte key gather.
// The mirror is a quarter of the keys' size, so its gathers hit the caches
// more often; the filter pays off once most vertices have been reached.
constexpr uint32_t kMirrorNone = 0xffffu;

template <bool FILTER>
struct SsspMark {
  const uint32_t* __restrict__ W;
  unsigned long long* __restrict__ keys;
  uint8_t* __restrict__ marks;
  const int32_t* __restrict__ perm;
  const uint16_t* __restrict__ mirror;

  using pay_t = int32_t;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return (int32_t)(uint32_t)(keys[u] >> 32);
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t e) const { return W[e]; }
  // the key test happens in commit_batch, whose loads are batched anyway
  __device__ __forceinline__ bool probe(int32_t, int32_t du, int32_t, uint32_t w) const {
    return (uint64_t)(uint32_t)du + (uint64_t)w < 0xffffffffull;
  }
  template <int B>
  __device__ __forceinline__ void commit_batch(const int32_t (&u)[B], const int32_t (&du)[B],
                                               const int32_t (&v)[B], const uint32_t (&w)[B],
                                               const bool (&ok)[B], int (&code)[B]) const {
    bool pass[B];
    if constexpr (FILTER) {
      uint32_t m[B];
#pragma unroll
      for (int r = 0; r < B; ++r) m[r] = ok[r] ? (uint32_t)mirror[v[r]] : 0u;
#pragma unroll
      for (int r = 0; r < B; ++r)
        pass[r] = ok[r] && (m[r] == kMirrorNone || (uint64_t)(uint32_t)du[r] + w[r] <= m[r]);
    } else {
#pragma unroll
      for (int r = 0; r < B; ++r) pass[r] = ok[r];
    }
    unsigned long long k[B];
#pragma unroll
    for (int r = 0; r < B; ++r) k[r] = pass[r] ? keys[v[r]] : 0ull;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      code[r] = 0;
      if (!pass[r]) continue;
      const uint64_t cand = (uint64_t)(uint32_t)du[r] + (uint64_t)w[r];
      const unsigned long long nk = (cand << 32) | caller_id(perm, u[r]);
      if (nk < k[r]) atomicMin(&keys[v[r]], nk);
      if (cand < (k[r] >> 32)) marks[v[r]] = 1;
    }
  }
  __device__ __forceinline__ bool commit(int32_t, int32_t, int32_t, uint32_t) const { return false; }
};

__device__ __forceinline__ uint16_t mirror_of(unsigned long long key) {
  const uint32_t d = (uint32_t)(key >> 32);
  return (uint16_t)(d < kMirrorNone ? d : kMirrorNone);
}

// Keys of the 32 consecutive vertices v0 .. v0 + 31 (v0 a multiple of 32, all
// below V), two per 16-byte load.  All loads are issued before any is used:
// loading only the marked ones (a loop over the set bits, or one branch per
// load) makes each wait for the previous one.
__device__ __forceinline__ void word_keys(const unsigned long long* __restrict__ keys, int64_t v0,
                                          unsigned long long (&k)[32]) {
  const ulonglong2* __restrict__ k2 = reinterpret_cast<const ulonglong2*>(keys + v0);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const ulonglong2 x = k2[j];
    k[2 * j] = x.x;
    k[2 * j + 1] = x.y;
  }
}

// One thread per 32 vertices: gather and clear the marks, list the marked
// vertices (ascending within each workgroup).
// The distance mirror of every marked vertex is refreshed on the way.
__global__ __launch_bounds__(256) void k_sssp_mark_compact(uint8_t* __restrict__ marks, int64_t V,
                                                           const unsigned long long* __restrict__ keys,
                                                           uint16_t* __restrict__ mirror,
                                                           int32_t* __restrict__ out_q,
                                                           uint32_t* __restrict__ out_count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t mask = take_marks(marks, w, V);
  const int64_t v0 = w * 32;
  if (mask && v0 + 32 <= V) {
    unsigned long long k[32];
    word_keys(keys, v0, k);
#pragma unroll
    for (int b = 0; b < 32; ++b)
      if ((mask >> b) & 1u) mirror[v0 + b] = mirror_of(k[b]);
  } else {
    for (uint32_t m = mask; m; m &= m - 1) {
      const int64_t v = v0 + __ffs(m) - 1;
      mirror[v] = mirror_of(keys[v]);
    }
  }
  append_mask<256>(mask, w, out_q, out_count);
}

// The same with the near / far split of the priority queue: a marked vertex
// whose distance is below the threshold T joins the next frontier, any other
// joins far pile fc unless it is already there in this generation (far_tag).
// Only the thread owning a vertex reads or writes its far tag here; the
// distance mirror is refreshed as in k_sssp_mark_compact.
__global__ __launch_bounds__(256) void k_sssp_pq_mark_compact(
    uint8_t* __restrict__ marks, int64_t V, const unsigned long long* __restrict__ keys,
    uint16_t* __restrict__ mirror, uint32_t T, int32_t epoch, int32_t* __restrict__ far_tag,
    int32_t* __restrict__ far_q,
    uint32_t* __restrict__ far_count, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t mask = take_marks(marks, w, V), near = 0, far = 0;
  const int64_t v0 = w * 32;
  if (mask && v0 + 32 <= V) {
    unsigned long long k[32];
    word_keys(keys, v0, k);
    int32_t ft[32];
    const int4* __restrict__ f4 = reinterpret_cast<const int4*>(far_tag + v0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int4 x = f4[j];
      ft[4 * j] = x.x;
      ft[4 * j + 1] = x.y;
      ft[4 * j + 2] = x.z;
      ft[4 * j + 3] = x.w;
    }
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      if (!((mask >> b) & 1u)) continue;
      mirror[v0 + b] = mirror_of(k[b]);
      if ((uint32_t)(k[b] >> 32) < T) {
        near |= 1u << b;
      } else if (ft[b] != epoch) {
        far_tag[v0 + b] = epoch;
        far |= 1u << b;
      }
    }
  } else {
    for (uint32_t m = mask; m; m &= m - 1) {
      const int b = __ffs(m) - 1;
      const int64_t v = v0 + b;
      const unsigned long long key = keys[v];
      mirror[v] = mirror_of(key);
      if ((uint32_t)(key >> 32) < T) {
        near |= 1u << b;
      } else if (far_tag[v] != epoch) {
        far_tag[v] = epoch;
        far |= 1u << b;
      }
    }
  }
  append_mask<256>(near, w, out_q, out_count);
  append_mask<256>(far, w, far_q, far_count);
}

__device__ __forceinline__ uint32_t pq_next_threshold(uint32_t T, uint32_t delta) {
  const uint64_t t = (uint64_t)T + delta;
  return t >= 0xffffffffull ? 0xffffffffu : (uint32_t)t;
}

// Split far pile fc into the next frontier and far pile (fc + 1) % 3 (see the
// file comment).  Grid-stride over kRefillItems entries per thread; both
// lists are appended with one atomic per workgroup and round, so every thread
// of the workgroup must call it.
constexpr int kRefillItems = 4;
__device__ __forceinline__ void pq_refill_pass(const unsigned long long* __restrict__ keys,
                                               uint32_t T, uint32_t delta, int32_t epoch, int32_t fc,
                                               int32_t* __restrict__ far_base,
                                               int32_t* __restrict__ far_tag, int64_t V, Ctrl* ctrl,
                                               int32_t* __restrict__ out_q, uint32_t* out_count) {
  constexpr int K = kRefillItems;
  const uint32_t T1 = pq_next_threshold(T, delta);
  const int32_t fn = (fc + 1) % 3;
  const int32_t* __restrict__ in = far_base + (int64_t)fc * V;
  int32_t* __restrict__ keep_q = far_base + (int64_t)fn * V;
  const int64_t n = ctrl->far_count[fc];
  const int64_t per_round = (int64_t)kAdvBlock * K;
  const int64_t stride = (int64_t)gridDim.x * per_round;
  for (int64_t base = (int64_t)blockIdx.x * per_round; base < n; base += stride) {
    int32_t v[K];
    bool near[K], keep[K];
    uint32_t n_near = 0, n_keep = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const int64_t i = base + r * kAdvBlock + threadIdx.x;
      v[r] = i < n ? in[i] : -1;
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const uint32_t d = v[r] >= 0 ? (uint32_t)(keys[v[r]] >> 32) : 0u;
      near[r] = v[r] >= 0 && d >= T && d < T1;
      keep[r] = v[r] >= 0 && d >= T1;
      if (keep[r]) far_tag[v[r]] = epoch + 1;
      n_near += near[r] ? 1u : 0u;
      n_keep += keep[r] ? 1u : 0u;
    }
    uint32_t s1 = block_append<kAdvBlock>(n_near, out_count);
    uint32_t s2 = block_append<kAdvBlock>(n_keep, &ctrl->far_count[fn]);
#pragma unroll
    for (int r = 0; r < K; ++r) {
      if (near[r]) out_q[s1++] = v[r];
      if (keep[r]) keep_q[s2++] = v[r];
    }
  }
}

struct SsspPqVisit {
  const uint32_t* __restrict__ W;
  unsigned long long* __restrict__ keys;
  int32_t* __restrict__ tags;
  int32_t next_tag;
  uint32_t T;
  uint32_t delta;
  int32_t epoch;
  int32_t fc;
  int32_t* __restrict__ far_base;
  int32_t* __restrict__ far_tag;
  int64_t V;
  int32_t* __restrict__ far_q;    // far_base + fc * V
  uint32_t* far_count;            // &ctrl->far_count[fc]
  const int32_t* __restrict__ perm;

  using pay_t = int32_t;
  static constexpr bool kFar = true;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return (int32_t)(uint32_t)(keys[u] >> 32);
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t e) const { return W[e]; }
  __device__ __forceinline__ bool probe(int32_t, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    if (cand >= 0xffffffffull) return false;
    return cand <= (keys[v] >> 32);
  }
  // 1: next frontier, 2: far pile, 0: nothing to append
  __device__ __forceinline__ int commit(int32_t u, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    const unsigned long long nk = (cand << 32) | caller_id(perm, u);
    const unsigned long long old = atomicMin(&keys[v], nk);
    if (cand >= (old >> 32)) return 0;
    if (cand < T) return atomicExch(&tags[v], next_tag) != next_tag ? 1 : 0;
    return atomicExch(&far_tag[v], epoch) != epoch ? 2 : 0;
  }
  template <int B>
  __device__ __forceinline__ void commit_batch(const int32_t (&u)[B], const int32_t (&du)[B],
                                               const int32_t (&v)[B], const uint32_t (&w)[B],
                                               const bool (&ok)[B], int (&code)[B]) const {
    unsigned long long nk[B];
    int32_t prev[B];
    bool imp[B];
#pragma unroll
    for (int r = 0; r < B; ++r)
      nk[r] = (((uint64_t)(uint32_t)du[r] + (uint64_t)w[r]) << 32) | (ok[r] ? caller_id(perm, u[r]) : 0u);
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const unsigned long long old = ok[r] ? atomicMin(&keys[v[r]], nk[r]) : 0ull;
      imp[r] = ok[r] && (nk[r] >> 32) < (old >> 32);
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const bool near = (nk[r] >> 32) < T;
      const int32_t val = near ? next_tag : epoch;
      prev[r] = imp[r] ? atomicExch(near ? &tags[v[r]] : &far_tag[v[r]], val) : val;
      code[r] = prev[r] != val ? (near ? 1 : 2) : 0;
    }
  }
  __device__ __forceinline__ void frontier_vertex(int32_t) const {}
  // device-predicated levels read the queue state of their step
  __device__ __forceinline__ SsspPqVisit prepare(Ctrl* ctrl, int step) const {
    SsspPqVisit g = *this;
    const int s = step & 1;
    g.T = ctrl->pq_T[s];
    g.epoch = ctrl->pq_epoch[s];
    g.fc = ctrl->pq_fc[s];
    g.far_q = far_base + (int64_t)g.fc * V;
    g.far_count = &ctrl->far_count[g.fc];
    return g;
  }
  // a refill step inside a device-predicated block runs on that block's small
  // grid, so only modest far piles are split there; larger ones end the block
  // and are split by the full-grid refill kernel
  __device__ __forceinline__ bool far_pending(const Ctrl* ctrl) const {
    const uint32_t n = ctrl->far_count[fc];
    return n > 0 && n <= kDlMaxRefill;
  }
  // queue state of the next step (called once, by one thread)
  __device__ __forceinline__ void advance(Ctrl* ctrl, int step, bool refill) const {
    const int s = (step + 1) & 1;
    if (refill) {
      ctrl->pq_T[s] = pq_next_threshold(T, delta);
      ctrl->pq_epoch[s] = epoch + 1;
      ctrl->pq_fc[s] = (fc + 1) % 3;
      ctrl->far_count[(fc + 2) % 3] = 0;  // the pile the next refill fills
    } else {
      ctrl->pq_T[s] = T;
      ctrl->pq_epoch[s] = epoch;
      ctrl->pq_fc[s] = fc;
    }
  }
  __device__ __forceinline__ void refill(Ctrl* ctrl, int32_t* out_q, uint32_t* out_count) const {
    pq_refill_pass(keys, T, delta, epoch, fc, far_base, far_tag, V, ctrl, out_q, out_count);
  }
};

__global__ __launch_bounds__(kAdvBlock) void k_sssp_pq_refill(const unsigned long long* __restrict__ keys,
                                                        PqState pq, Ctrl* __restrict__ ctrl,
                                                        int32_t* __restrict__ out_q,
                                                        uint32_t* __restrict__ out_count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->far_count[(pq.fc + 2) % 3] = 0;
  pq_refill_pass(keys, pq.T, pq.delta, pq.epoch, pq.fc, pq.far_base, pq.far_tag, pq.V, ctrl, out_q,
                 out_count);
}

__global__ __launch_bounds__(256) void k_sssp_init(unsigned long long* __restrict__ keys,
                                                   int32_t* __restrict__ tags,
                                                   int32_t* __restrict__ far_tag,
                                                   uint16_t* __restrict__ mirror, int64_t V,
                                                   Ctrl* __restrict__ ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
    keys[v] = ~0ull;
    tags[v] = -1;
    if (far_tag) far_tag[v] = -1;
    mirror[v] = (uint16_t)kMirrorNone;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->far_count[0] = ctrl->far_count[1] = ctrl->far_count[2] = 0;
    ctrl->q_count[1] = 0;
    ctrl->q_count[2] = 0;
    ctrl->inspected = 0;
    ctrl->reached_edges = 0;
    ctrl->m_f[0] = ctrl->m_f[1] = 0;
    ctrl->max_deg[0] = ctrl->max_deg[1] = 0;
  }
}

// Sources: distance 0, no predecessor; the deduplicated list is frontier 0.
__global__ __launch_bounds__(256) void k_sssp_seed(const int32_t* __restrict__ src, int32_t n,
                                                   unsigned long long* __restrict__ keys,
                                                   int32_t* __restrict__ tags,
                                                   Ctrl* __restrict__ ctrl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    keys[src[i]] = 0xffffffffull;
    tags[src[i]] = 0;
  }
  if (i == 0) ctrl->q_count[0] = (uint32_t)n;
}

__global__ __launch_bounds__(256) void k_sssp_finalize(const unsigned long long* __restrict__ keys,
                                                       const int32_t* __restrict__ R, int64_t V,
                                                       uint32_t* __restrict__ dist,
                                                       int32_t* __restrict__ pred,
                                                       const int32_t* __restrict__ perm,
                                                       int64_t* __restrict__ reached_edges) {
  __shared__ int64_t s[256 / kWave];
  // kFinalItems vertices per thread and round, all loaded before any is used
  // (past V the loads repeat vertex V - 1 and the results are dropped)
  constexpr int kFinalItems = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t acc = 0;
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < V;
       v0 += stride * kFinalItems) {
    unsigned long long k[kFinalItems];
    int32_t a[kFinalItems], b[kFinalItems], o[kFinalItems];
#pragma unroll
    for (int r = 0; r < kFinalItems; ++r) {
      const int64_t v = v0 + r * stride < V ? v0 + r * stride : V - 1;
      k[r] = keys[v];
      a[r] = R[v];
      b[r] = R[v + 1];
      o[r] = perm ? perm[v] : (int32_t)v;
    }
#pragma unroll
    for (int r = 0; r < kFinalItems; ++r) {
      if (v0 + r * stride >= V) continue;
      const uint32_t d = (uint32_t)(k[r] >> 32);
      dist[o[r]] = d;
      if (pred) pred[o[r]] = (int32_t)(uint32_t)(k[r] & 0xffffffffull);
      if (d != 0xffffffffu) acc += (int64_t)b[r] - a[r];
    }
  }
  acc = wave_sum(acc);
  if (lane() == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < 256 / kWave; ++i) t += s[i];
    atomicAdd((unsigned long long*)reached_edges, (unsigned long long)t);
  }
}

// Sources have no predecessor even where a zero-weight edge ties them.
__global__ __launch_bounds__(256) void k_sssp_source_pred(const int32_t* __restrict__ src,
                                                          int32_t n, int32_t* __restrict__ pred) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pred[src[i]] = -1;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_sssp_init(unsigned long long* keys, int32_t* tags, int32_t* far_tag,
                            uint16_t* mirror, int64_t V, Ctrl* ctrl, hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 4096) g = 4096;
  k_sssp_init<<<g, 256, 0, st>>>(keys, tags, far_tag, mirror, V, ctrl);
  return hipGetLastError();
}

hipError_t launch_sssp_seed(const int32_t* src_dev, int32_t n, unsigned long long* keys,
                            int32_t* tags, Ctrl* ctrl, hipStream_t st) {
  k_sssp_seed<<<blocks_for(n, 256), 256, 0, st>>>(src_dev, n, keys, tags, ctrl);
  return hipGetLastError();
}

hipError_t launch_sssp_relax(int mode, const int32_t* frontier, const int32_t* offsets,
                             const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                             int64_t m_f, const int32_t* R, const int32_t* C, const uint32_t* W,
                             unsigned long long* keys, int32_t* tags, const int32_t* perm,
                             int32_t next_tag, int32_t* out_q, uint32_t* out_count, const AdvCfg& cfg,
                             hipStream_t st) {
  SsspVisit f{W, keys, tags, perm, next_tag};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, out_q,
                       out_count, cfg, st);
}

hipError_t launch_sssp_finalize(const unsigned long long* keys, const int32_t* R, int64_t V,
                                uint32_t* dist, int32_t* pred, const int32_t* perm,
                                const int32_t* src_orig_dev, int32_t n_src, int64_t* reached_edges,
                                hipStream_t st) {
  // grid-stride, one atomic per workgroup for the reached-edge sum: a modest
  // grid keeps those atomics (all on one address) few
  unsigned g = blocks_for(V, 256);
  if (g > 1024) g = 1024;
  k_sssp_finalize<<<g, 256, 0, st>>>(keys, R, V, dist, pred, perm, reached_edges);
  if (pred)
    k_sssp_source_pred<<<blocks_for(n_src, 256), 256, 0, st>>>(src_orig_dev, n_src, pred);
  return hipGetLastError();
}

hipError_t launch_sssp_dstep(const DlArgs& a, const uint32_t* W, unsigned long long* keys,
                             int32_t* tags, const int32_t* perm, int32_t next_tag, int n_blocks,
                             hipStream_t st) {
  const SsspVisit f{W, keys, tags, perm, next_tag};
  k_dstep<SsspVisit><<<n_blocks, kAdvBlock, 0, st>>>(a, f);
  return hipGetLastError();
}

namespace {
SsspPqVisit pq_functor(const uint32_t* W, unsigned long long* keys, int32_t* tags, int32_t next_tag,
                       const PqState& pq, Ctrl* ctrl) {
  return SsspPqVisit{W,          keys,     tags,          next_tag,
                     pq.T,       pq.delta, pq.epoch,      pq.fc,
                     pq.far_base, pq.far_tag, pq.V,     pq.far_base + (int64_t)pq.fc * pq.V,
                     &ctrl->far_count[pq.fc], pq.perm};
}
}  // namespace

hipError_t launch_sssp_pq_relax(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C, const uint32_t* W,
                                unsigned long long* keys, int32_t* tags, int32_t next_tag,
                                const PqState& pq, Ctrl* ctrl, int32_t* out_q, uint32_t* out_count,
                                const AdvCfg& cfg, hipStream_t st) {
  const SsspPqVisit f = pq_functor(W, keys, tags, next_tag, pq, ctrl);
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, out_q,
                       out_count, cfg, st);
}

hipError_t launch_sssp_pq_refill(const unsigned long long* keys, const PqState& pq, Ctrl* ctrl,
                                 int64_t max_n, int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  unsigned g = blocks_for(max_n > 0 ? max_n : 1, kAdvBlock * kRefillItems);
  if (g > 4096) g = 4096;
  k_sssp_pq_refill<<<g, kAdvBlock, 0, st>>>(keys, pq, ctrl, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_sssp_pq_dstep(const DlArgs& a, const uint32_t* W, unsigned long long* keys,
                                int32_t* tags, int32_t next_tag, const PqState& pq, int n_blocks,
                                hipStream_t st) {
  const SsspPqVisit f = pq_functor(W, keys, tags, next_tag, pq, a.ctrl);
  k_dstep<SsspPqVisit><<<n_blocks, kAdvBlock, 0, st>>>(a, f);
  return hipGetLastError();
}

hipError_t launch_sssp_relax_marks(int mode, const int32_t* frontier, const int32_t* offsets,
                                   const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                   int64_t m_f, const int32_t* R, const int32_t* C,
                                   const uint32_t* W, unsigned long long* keys,
                                   const int32_t* perm, uint8_t* marks, const uint16_t* mirror,
                                   bool filter, const AdvCfg& cfg, hipStream_t st) {
  if (filter) {
    const SsspMark<true> f{W, keys, marks, perm, mirror};
    return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                         nullptr, cfg, st);
  }
  const SsspMark<false> f{W, keys, marks, perm, mirror};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st);
}

hipError_t launch_sssp_pq_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                       uint16_t* mirror, const PqState& pq, Ctrl* ctrl,
                                       int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  if (n_words <= 0) return hipSuccess;
  k_sssp_pq_mark_compact<<<blocks_for(n_words, 256), 256, 0, st>>>(
      marks, V, keys, mirror, pq.T, pq.epoch, pq.far_tag, pq.far_base + (int64_t)pq.fc * pq.V,
      &ctrl->far_count[pq.fc], out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_sssp_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                    uint16_t* mirror, int32_t* out_q, uint32_t* out_count,
                                    hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  if (n_words <= 0) return hipSuccess;
  k_sssp_mark_compact<<<blocks_for(n_words, 256), 256, 0, st>>>(marks, V, keys, mirror, out_q,
                                                                out_count);
  return hipGetLastError();
}

}  // namespace gr
