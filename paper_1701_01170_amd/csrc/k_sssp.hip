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
// With FILTER, a one-byte distance mirror (ceil(dist / 2^shift) of an
// earlier moment, 255 when unknown or too large; refreshed by the compaction
// for every marked vertex) screens the edges first.  Distances only decrease,
// so a mirror value m below 255 bounds the current distance by m * 2^shift: an
// edge whose candidate exceeds that can neither shorten the distance nor tie
// it, and skips the 8-byte key gather.  The mirror is an eighth of the keys'
// size, so its gathers hit the caches more often; the filter pays off once
// most vertices have been reached.  The quantum 2^shift is chosen per graph
// so that 254 steps cover about four times its largest weight.
//
// With `relaxed` (nullable), every chunk that stages a frontier vertex u
// raises relaxed[u] to 1 + the distance it relaxes u's edges with; the
// compaction resets relaxed[] to 0 for the vertices it lets into the next
// frontier.  Distances only decrease, so after an iteration relaxed[v] equals
// dist(v) + 1 exactly when v was in the frontier and every chunk of its row
// already read its final distance: its edges went out with that distance, and
// the compaction drops v from the next frontier (Remove_Redundant applied to
// work already done).  A value left from an earlier iteration is larger than
// 1 + any distance v can have after dropping in this one, and 0 never
// matches, so nothing else is dropped.
constexpr uint32_t kMirrorNone = 0xffu;

template <bool FILTER>
struct SsspMark {
  const uint32_t* __restrict__ W;
  unsigned long long* __restrict__ keys;
  uint8_t* __restrict__ marks;
  const int32_t* __restrict__ perm;
  DistMirror mirror;
  uint32_t* __restrict__ relaxed;  // nullable

  using pay_t = int32_t;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = true;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return (int32_t)(uint32_t)(keys[u] >> 32);
  }
  // a frontier vertex's distance is below UINT32_MAX, so du + 1 does not wrap
  __device__ __forceinline__ void seg_note(int32_t u, int32_t du) const {
    if (relaxed) atomicMax(&relaxed[u], (uint32_t)du + 1u);
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
      for (int r = 0; r < B; ++r) m[r] = ok[r] ? (uint32_t)mirror.p[v[r]] : 0u;
#pragma unroll
      for (int r = 0; r < B; ++r)
        pass[r] = ok[r] && (m[r] == kMirrorNone ||
                            (uint64_t)(uint32_t)du[r] + w[r] <= ((uint64_t)m[r] << mirror.shift));
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

// mirror entry of a vertex with this key: ceil(dist / 2^shift), or 255
__device__ __forceinline__ uint8_t mirror_of(unsigned long long key, uint32_t shift) {
  const uint64_t d = key >> 32;
  const uint64_t q = (d + ((1ull << shift) - 1ull)) >> shift;
  return (uint8_t)(q < kMirrorNone ? q : kMirrorNone);
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

// relaxed[] of the 32 consecutive vertices v0 .. v0 + 31 (v0 a multiple of
// 32, all below V), four per 16-byte load.
__device__ __forceinline__ void word_relaxed(const uint32_t* __restrict__ relaxed, int64_t v0,
                                             uint32_t (&r)[32]) {
  const uint4* __restrict__ r4 = reinterpret_cast<const uint4*>(relaxed + v0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint4 x = r4[j];
    r[4 * j] = x.x;
    r[4 * j + 1] = x.y;
    r[4 * j + 2] = x.z;
    r[4 * j + 3] = x.w;
  }
}

// Whether marked vertex v (key k, relaxed value r) stays out of the next
// frontier; otherwise its relaxed[] entry is reset for the iteration it joins.
__device__ __forceinline__ bool drop_relaxed(uint32_t* __restrict__ relaxed, int64_t v,
                                             unsigned long long k, uint32_t r) {
  if (r == (uint32_t)(k >> 32) + 1u) return true;
  if (r != 0u) relaxed[v] = 0u;
  return false;
}

// One thread per 32 vertices: gather and clear the marks, list the marked
// vertices (ascending within each workgroup), except those whose edges this
// iteration already relaxed with their final distance (relaxed, nullable).
// The distance mirror of every marked vertex is refreshed on the way.
__global__ __launch_bounds__(256) void k_sssp_mark_compact(uint8_t* __restrict__ marks, int64_t V,
                                                           const unsigned long long* __restrict__ keys,
                                                           DistMirror mirror,
                                                           uint32_t* __restrict__ relaxed,
                                                           int32_t* __restrict__ out_q,
                                                           uint32_t* __restrict__ out_count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t mask = take_marks(marks, w, V);
  const int64_t v0 = w * 32;
  if (mask && v0 + 32 <= V) {
    unsigned long long k[32];
    word_keys(keys, v0, k);
    if (relaxed) {
      uint32_t r[32];
      word_relaxed(relaxed, v0, r);
#pragma unroll
      for (int b = 0; b < 32; ++b) {
        if (!((mask >> b) & 1u)) continue;
        mirror.p[v0 + b] = mirror_of(k[b], mirror.shift);
        if (drop_relaxed(relaxed, v0 + b, k[b], r[b])) mask &= ~(1u << b);
      }
    } else {
#pragma unroll
      for (int b = 0; b < 32; ++b)
        if ((mask >> b) & 1u) mirror.p[v0 + b] = mirror_of(k[b], mirror.shift);
    }
  } else {
    for (uint32_t m = mask; m; m &= m - 1) {
      const int b = __ffs(m) - 1;
      const int64_t v = v0 + b;
      const unsigned long long key = keys[v];
      mirror.p[v] = mirror_of(key, mirror.shift);
      if (relaxed && drop_relaxed(relaxed, v, key, relaxed[v])) mask &= ~(1u << b);
    }
  }
  append_mask<256>(mask, w, out_q, out_count);
}

// Distance-ordered compaction (without the priority queue).  Vertices are
// relaxed roughly in frontier order (workgroups start in chunk order), so a
// frontier that lists small distances first lets their improvements reach the
// larger-distance vertices before those are staged: fewer edges go out with
// a distance that later drops (Sec. 5.1: the priority queue's aim, without its
// extra iterations).  The marked vertices are binned by
// (dist - base) >> shift into kSsspBins bins (the last takes everything
// beyond), where base is a lower bound of every distance the iteration can
// have produced: the lower edge of the previous binned frontier's first
// non-empty bin (distances assigned in an iteration are at least the
// smallest distance of its frontier).  Pass 1 culls, refreshes the mirror,
// writes bin + 1 into the mark byte and counts bins per workgroup into one of
// kBinCopies histograms; the scan lays the bins out (copies of a bin in
// order) and moves base; pass 2, on the same grid, scatters each vertex into
// its bin's range (order inside a bin: by workgroup, then arbitrary).
__device__ __forceinline__ uint32_t peek_marks(const uint8_t* __restrict__ marks, int64_t w,
                                               int64_t V, uint8_t (&m)[32]) {
  const int64_t v0 = w * 32;
  uint32_t mask = 0;
  if (v0 + 32 <= V) {
    const uint4* m4 = reinterpret_cast<const uint4*>(marks + v0);
    const uint4 a = m4[0], b = m4[1];
    const uint32_t q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        m[4 * i + k] = (uint8_t)(q[i] >> (8 * k));
        if (m[4 * i + k]) mask |= 1u << (4 * i + k);
      }
  } else {
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      m[b] = v0 + b < V ? marks[v0 + b] : (uint8_t)0;
      if (m[b]) mask |= 1u << b;
    }
  }
  return mask;
}

__device__ __forceinline__ void put_marks(uint8_t* __restrict__ marks, int64_t w, int64_t V,
                                          const uint8_t (&m)[32]) {
  const int64_t v0 = w * 32;
  if (v0 + 32 <= V) {
    uint32_t q[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      q[i] = (uint32_t)m[4 * i] | ((uint32_t)m[4 * i + 1] << 8) | ((uint32_t)m[4 * i + 2] << 16) |
             ((uint32_t)m[4 * i + 3] << 24);
    uint4* z = reinterpret_cast<uint4*>(marks + v0);
    z[0] = make_uint4(q[0], q[1], q[2], q[3]);
    z[1] = make_uint4(q[4], q[5], q[6], q[7]);
  } else {
    for (int b = 0; b < 32 && v0 + b < V; ++b) marks[v0 + b] = m[b];
  }
}

__device__ __forceinline__ uint32_t dist_bin(uint32_t d, uint32_t base, uint32_t shift) {
  const uint32_t x = d > base ? (d - base) >> shift : 0u;
  return x < (uint32_t)kSsspBins ? x : (uint32_t)kSsspBins - 1u;
}

__global__ __launch_bounds__(256) void k_sssp_bin_count(uint8_t* __restrict__ marks, int64_t V,
                                                        const unsigned long long* __restrict__ keys,
                                                        DistMirror mirror,
                                                        uint32_t* __restrict__ relaxed,
                                                        SsspBins bins) {
  __shared__ uint32_t s_h[kSsspBins];
  for (int i = threadIdx.x; i < kSsspBins; i += 256) s_h[i] = 0;
  __syncthreads();
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t base = bins.state[kSsspBinBase];
  uint8_t m[32];
  const uint32_t mask = w < (V + 31) / 32 ? peek_marks(marks, w, V, m) : 0u;
  if (mask) {
    const int64_t v0 = w * 32;
    unsigned long long k[32];
    uint32_t r[32];
    if (v0 + 32 <= V) {
      word_keys(keys, v0, k);
      if (relaxed) word_relaxed(relaxed, v0, r);
    } else {
#pragma unroll
      for (int b = 0; b < 32; ++b) {
        const bool in = (mask >> b) & 1u;
        k[b] = in ? keys[v0 + b] : 0ull;
        r[b] = in && relaxed ? relaxed[v0 + b] : 0u;
      }
    }
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      if (!((mask >> b) & 1u)) continue;
      mirror.p[v0 + b] = mirror_of(k[b], mirror.shift);
      if (relaxed && drop_relaxed(relaxed, v0 + b, k[b], r[b])) {
        m[b] = 0;
        continue;
      }
      const uint32_t bin = dist_bin((uint32_t)(k[b] >> 32), base, bins.shift);
      m[b] = (uint8_t)(bin + 1u);
      atomicAdd(&s_h[bin], 1u);
    }
    put_marks(marks, w, V, m);
  }
  __syncthreads();
  uint32_t* h = bins.state + kSsspBinHist + (blockIdx.x % kBinCopies) * kSsspBins;
  for (int i = threadIdx.x; i < kSsspBins; i += 256)
    if (s_h[i]) atomicAdd(&h[i], s_h[i]);
}

// One workgroup of kSsspBins threads: bin ranges (cursor of copy c of bin b =
// start of bin b + the counts of copies before c), the histograms cleared,
// the next base, and the frontier size.
__global__ __launch_bounds__(kSsspBins) void k_sssp_bin_scan(SsspBins bins,
                                                             uint32_t* __restrict__ out_count) {
  __shared__ uint32_t s_tmp[kSsspBins / kWave];
  __shared__ uint32_t s_first;
  const int b = threadIdx.x;
  uint32_t* h = bins.state + kSsspBinHist;
  uint32_t* cur = bins.state + kSsspBinCursor;
  uint32_t c[kBinCopies];
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < kBinCopies; ++i) {
    c[i] = h[i * kSsspBins + b];
    tot += c[i];
  }
  if (b == 0) s_first = kSsspBins;
  const uint32_t inc = wave_incl_scan(tot);
  if (lane() == kWave - 1) s_tmp[b / kWave] = inc;
  __syncthreads();
  if (tot) atomicMin(&s_first, (uint32_t)b);
  uint32_t start = inc - tot;
  for (int i = 0; i < b / kWave; ++i) start += s_tmp[i];
#pragma unroll
  for (int i = 0; i < kBinCopies; ++i) {
    cur[i * kSsspBins + b] = start;
    start += c[i];
    h[i * kSsspBins + b] = 0u;
  }
  __syncthreads();
  if (b == kSsspBins - 1) {
    *out_count = start;
    const uint32_t f = s_first;
    if (f < (uint32_t)kSsspBins) bins.state[kSsspBinBase] += f << bins.shift;
  }
}

__global__ __launch_bounds__(256) void k_sssp_bin_scatter(uint8_t* __restrict__ marks, int64_t V,
                                                          SsspBins bins,
                                                          int32_t* __restrict__ out_q) {
  __shared__ uint32_t s_n[kSsspBins];
  for (int i = threadIdx.x; i < kSsspBins; i += 256) s_n[i] = 0;
  __syncthreads();
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  uint8_t m[32];
  const uint32_t mask = w < (V + 31) / 32 ? peek_marks(marks, w, V, m) : 0u;
  uint32_t rank[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) rank[b] = (mask >> b) & 1u ? atomicAdd(&s_n[m[b] - 1], 1u) : 0u;
  if (mask) {
    uint8_t z[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) z[b] = 0;
    put_marks(marks, w, V, z);
  }
  __syncthreads();
  uint32_t* cur = bins.state + kSsspBinCursor + (blockIdx.x % kBinCopies) * kSsspBins;
  for (int i = threadIdx.x; i < kSsspBins; i += 256)
    if (s_n[i]) s_n[i] = atomicAdd(&cur[i], s_n[i]);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 32; ++b)
    if ((mask >> b) & 1u) out_q[s_n[m[b] - 1] + rank[b]] = (int32_t)(w * 32 + b);
}

// The same with the near / far split of the priority queue: a marked vertex
// whose distance is below the threshold T joins the next frontier, any other
// joins far pile fc unless it is already there in this generation (far_tag).
// Only the thread owning a vertex reads or writes its far tag here; the
// distance mirror is refreshed and vertices already relaxed with their final
// distance are dropped as in k_sssp_mark_compact.
__global__ __launch_bounds__(256) void k_sssp_pq_mark_compact(
    uint8_t* __restrict__ marks, int64_t V, const unsigned long long* __restrict__ keys,
    DistMirror mirror, uint32_t* __restrict__ relaxed, uint32_t T, int32_t epoch,
    int32_t* __restrict__ far_tag, int32_t* __restrict__ far_q,
    uint32_t* __restrict__ far_count, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t mask = take_marks(marks, w, V), near = 0, far = 0;
  const int64_t v0 = w * 32;
  if (mask && v0 + 32 <= V) {
    unsigned long long k[32];
    word_keys(keys, v0, k);
    uint32_t rl[32];
    if (relaxed) word_relaxed(relaxed, v0, rl);
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
      mirror.p[v0 + b] = mirror_of(k[b], mirror.shift);
      if (relaxed && drop_relaxed(relaxed, v0 + b, k[b], rl[b])) continue;
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
      mirror.p[v] = mirror_of(key, mirror.shift);
      if (relaxed && drop_relaxed(relaxed, v, key, relaxed[v])) continue;
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
                                                   DistMirror mirror,
                                                   uint32_t* __restrict__ relaxed,
                                                   uint32_t* __restrict__ bin_state, int64_t V,
                                                   Ctrl* __restrict__ ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (bin_state && blockIdx.x == 0)
    for (int i = threadIdx.x; i < kSsspBinWords; i += blockDim.x) bin_state[i] = 0u;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
    keys[v] = ~0ull;
    tags[v] = -1;
    if (far_tag) far_tag[v] = -1;
    mirror.p[v] = (uint8_t)kMirrorNone;
    if (relaxed) relaxed[v] = 0u;
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

// dist / pred at caller ids c and the degree sum of the reached vertices.
// With inv (renumbered graphs: caller id -> traversal id) the loop runs over
// caller ids: the key is gathered, the outputs written in order and the
// degree taken from the caller's row offsets (R_orig); scattering the outputs
// to perm[v] instead took 73 us per R-MAT 22 SSSP against 26 us in order.
__global__ __launch_bounds__(256) void k_sssp_finalize(const unsigned long long* __restrict__ keys,
                                                       const int32_t* __restrict__ R, int64_t V,
                                                       uint32_t* __restrict__ dist,
                                                       int32_t* __restrict__ pred,
                                                       const int32_t* __restrict__ inv,
                                                       int64_t* __restrict__ reached_edges) {
  __shared__ int64_t s[256 / kWave];
  // kFinalItems vertices per thread and round, all loaded before any is used
  // (past V the loads repeat vertex V - 1 and the results are dropped)
  constexpr int kFinalItems = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t acc = 0;
  for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c0 < V;
       c0 += stride * kFinalItems) {
    unsigned long long k[kFinalItems];
    int32_t a[kFinalItems], b[kFinalItems], v[kFinalItems];
#pragma unroll
    for (int r = 0; r < kFinalItems; ++r) {
      const int64_t c = c0 + r * stride < V ? c0 + r * stride : V - 1;
      v[r] = inv ? inv[c] : (int32_t)c;
      a[r] = R[c];  // R is the caller's row offsets when inv is given
      b[r] = R[c + 1];
    }
#pragma unroll
    for (int r = 0; r < kFinalItems; ++r) k[r] = keys[v[r]];
#pragma unroll
    for (int r = 0; r < kFinalItems; ++r) {
      const int64_t c = c0 + r * stride;
      if (c >= V) continue;
      const uint32_t d = (uint32_t)(k[r] >> 32);
      dist[c] = d;
      if (pred) pred[c] = (int32_t)(uint32_t)(k[r] & 0xffffffffull);
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
                            DistMirror mirror, uint32_t* relaxed, uint32_t* bin_state, int64_t V,
                            Ctrl* ctrl, hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 4096) g = 4096;
  k_sssp_init<<<g, 256, 0, st>>>(keys, tags, far_tag, mirror, relaxed, bin_state, V, ctrl);
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
                                uint32_t* dist, int32_t* pred, const int32_t* inv,
                                const int32_t* src_orig_dev, int32_t n_src, int64_t* reached_edges,
                                hipStream_t st) {
  // grid-stride, one atomic per workgroup for the reached-edge sum: a modest
  // grid keeps those atomics (all on one address) few
  unsigned g = blocks_for(V, 256);
  if (g > 1024) g = 1024;
  k_sssp_finalize<<<g, 256, 0, st>>>(keys, R, V, dist, pred, inv, reached_edges);
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
                                   const int32_t* perm, uint8_t* marks, const DistMirror mirror,
                                   uint32_t* relaxed, bool filter, const AdvCfg& cfg,
                                   hipStream_t st) {
  if (filter) {
    const SsspMark<true> f{W, keys, marks, perm, mirror, relaxed};
    return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                         nullptr, cfg, st);
  }
  const SsspMark<false> f{W, keys, marks, perm, mirror, relaxed};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st);
}

hipError_t launch_sssp_pq_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                       DistMirror mirror, uint32_t* relaxed, const PqState& pq,
                                       Ctrl* ctrl, int32_t* out_q, uint32_t* out_count,
                                       hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  if (n_words <= 0) return hipSuccess;
  k_sssp_pq_mark_compact<<<blocks_for(n_words, 256), 256, 0, st>>>(
      marks, V, keys, mirror, relaxed, pq.T, pq.epoch, pq.far_tag, pq.far_base + (int64_t)pq.fc * pq.V,
      &ctrl->far_count[pq.fc], out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_sssp_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                    DistMirror mirror, uint32_t* relaxed, int32_t* out_q,
                                    uint32_t* out_count, hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  if (n_words <= 0) return hipSuccess;
  k_sssp_mark_compact<<<blocks_for(n_words, 256), 256, 0, st>>>(marks, V, keys, mirror, relaxed,
                                                                out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_sssp_bin_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                   DistMirror mirror, uint32_t* relaxed, const SsspBins& bins,
                                   int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  const int64_t n_words = (V + 31) / 32;
  if (n_words <= 0) return hipSuccess;
  const unsigned g = blocks_for(n_words, 256);
  k_sssp_bin_count<<<g, 256, 0, st>>>(marks, V, keys, mirror, relaxed, bins);
  k_sssp_bin_scan<<<1, kSsspBins, 0, st>>>(bins, out_count);
  k_sssp_bin_scatter<<<g, 256, 0, st>>>(marks, V, bins, out_q);
  return hipGetLastError();
}

}  // namespace gr
