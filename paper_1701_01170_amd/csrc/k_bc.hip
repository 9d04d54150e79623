// Betweenness centrality (Sec. 6, betweenness centrality; Brandes's two
// passes) on the advance operator.  The forward pass is the BFS (depths) and
// then, level by level, a push advance over each level's vertices that adds
// sigma(u) into sigma(w) for every edge (u, w) into the next level; the
// backward pass walks the levels in reverse, each a push advance over the
// level's vertices w that adds 1 / sigma(w) + acc(w) into acc(v) for every edge
// (w, v) into the level before, where acc(v) = sum over v's successors w of
// (1 + delta(w)) / sigma(w), so delta(v) = sigma(v) * acc(v) and the payload
// (1 + delta(w)) / sigma(w) equals 1 / sigma(w) + acc(w).  The edges of a
// level are balanced by the same TWC / LB kernels as the traversals; the
// per-vertex sums use hardware fp64 atomic adds on the targets (device memory
// from hipMalloc, coarse grained).  Levels come from a counting sort of the
// depths, so every level's vertices are contiguous.
#include "k_advance.h"

namespace gr {

namespace {

struct BcSigma {
  const int32_t* __restrict__ depth;
  double* __restrict__ sigma;
  int32_t next_depth;

  using pay_t = double;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = false;
  __device__ __forceinline__ double seg_payload(int32_t u) const { return sigma[u]; }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ bool probe(int32_t, double, int32_t w, uint32_t) const {
    return depth[w] == next_depth;
  }
  __device__ __forceinline__ bool commit(int32_t, double s, int32_t w, uint32_t) const {
    unsafeAtomicAdd(&sigma[w], s);
    return false;
  }
};

struct BcDependency {
  const int32_t* __restrict__ depth;
  const double* __restrict__ sigma;
  double* __restrict__ acc;
  int32_t prev_depth;

  using pay_t = double;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = false;
  __device__ __forceinline__ double seg_payload(int32_t w) const {
    return 1.0 / sigma[w] + acc[w];
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ bool probe(int32_t, double, int32_t v, uint32_t) const {
    return depth[v] == prev_depth;
  }
  __device__ __forceinline__ bool commit(int32_t, double x, int32_t v, uint32_t) const {
    unsafeAtomicAdd(&acc[v], x);
    return false;
  }
};

constexpr int kBcBlock = 256;
constexpr int kBcItems = 8;            // vertices per thread per tile
constexpr int kBcLdsLevels = 4096;     // levels counted in LDS (more: global atomics)

// Vertices per level and their degree sums; sigma / acc initialised
// (sigma(source) = 1).  With at most kBcLdsLevels levels each workgroup
// counts its tile in LDS and adds its non-zero bins to the global counts.
__global__ __launch_bounds__(kBcBlock) void k_bc_level_count(
    const int32_t* __restrict__ depth, const int32_t* __restrict__ R, int64_t V, int32_t source,
    int32_t n_levels, uint32_t* __restrict__ lvl_n, unsigned long long* __restrict__ lvl_m,
    double* __restrict__ sigma, double* __restrict__ acc) {
  __shared__ uint32_t s_n[kBcLdsLevels];
  __shared__ unsigned long long s_m[kBcLdsLevels];
  const bool lds = n_levels <= kBcLdsLevels;
  if (lds) {
    for (int i = threadIdx.x; i < n_levels; i += kBcBlock) {
      s_n[i] = 0;
      s_m[i] = 0;
    }
    __syncthreads();
  }
  const int64_t tile = (int64_t)kBcBlock * kBcItems;
  const int64_t v0 = (int64_t)blockIdx.x * tile;
  for (int r = 0; r < kBcItems; ++r) {
    const int64_t v = v0 + (int64_t)r * kBcBlock + threadIdx.x;
    if (v >= V) break;
    const int32_t d = depth[v];
    sigma[v] = v == source ? 1.0 : 0.0;
    acc[v] = 0.0;
    if (d < 0 || d >= n_levels) continue;
    const unsigned long long deg = (unsigned long long)(R[v + 1] - R[v]);
    if (lds) {
      atomicAdd(&s_n[d], 1u);
      if (deg) atomicAdd(&s_m[d], deg);
    } else {
      atomicAdd(&lvl_n[d], 1u);
      if (deg) atomicAdd(&lvl_m[d], deg);
    }
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < n_levels; i += kBcBlock) {
      if (s_n[i]) atomicAdd(&lvl_n[i], s_n[i]);
      if (s_m[i]) atomicAdd(&lvl_m[i], s_m[i]);
    }
  }
}

// Scatter every reached vertex to its level's range of `levels` (cursor[d]
// starts at the level's offset).  With at most kBcLdsLevels levels a
// workgroup ranks its tile's vertices per level in LDS and reserves each
// level's range with one global atomic.
__global__ __launch_bounds__(kBcBlock) void k_bc_level_scatter(
    const int32_t* __restrict__ depth, int64_t V, int32_t n_levels,
    uint32_t* __restrict__ cursor, int32_t* __restrict__ levels) {
  __shared__ uint32_t s_n[kBcLdsLevels];
  const bool lds = n_levels <= kBcLdsLevels;
  const int64_t tile = (int64_t)kBcBlock * kBcItems;
  const int64_t v0 = (int64_t)blockIdx.x * tile;
  int32_t d[kBcItems];
  uint32_t rank[kBcItems];
  if (lds) {
    for (int i = threadIdx.x; i < n_levels; i += kBcBlock) s_n[i] = 0;
    __syncthreads();
  }
  for (int r = 0; r < kBcItems; ++r) {
    const int64_t v = v0 + (int64_t)r * kBcBlock + threadIdx.x;
    d[r] = v < V ? depth[v] : -1;
    if (d[r] >= n_levels) d[r] = -1;
    rank[r] = 0;
    if (d[r] >= 0) rank[r] = lds ? atomicAdd(&s_n[d[r]], 1u) : atomicAdd(&cursor[d[r]], 1u);
  }
  if (lds) {
    __syncthreads();
    // each non-empty bin reserves its range; s_n then holds the range base
    for (int i = threadIdx.x; i < n_levels; i += kBcBlock) {
      const uint32_t c = s_n[i];
      if (c) s_n[i] = atomicAdd(&cursor[i], c);
    }
    __syncthreads();
  }
  for (int r = 0; r < kBcItems; ++r) {
    if (d[r] < 0) continue;
    const int64_t v = v0 + (int64_t)r * kBcBlock + threadIdx.x;
    levels[lds ? s_n[d[r]] + rank[r] : rank[r]] = (int32_t)v;
  }
}

// bc(v) += delta(v) = sigma(v) * acc(v) for reached v != source; sigma out
// (nullable) for the caller.  Outputs at caller ids (perm nullable).
__global__ __launch_bounds__(kBcBlock) void k_bc_finalize(
    const int32_t* __restrict__ depth, const double* __restrict__ sigma,
    const double* __restrict__ acc, int64_t V, int32_t source, const int32_t* __restrict__ perm,
    double* __restrict__ bc, double* __restrict__ sigma_out) {
  const int64_t v = (int64_t)blockIdx.x * kBcBlock + threadIdx.x;
  if (v >= V) return;
  const int32_t c = perm ? perm[v] : (int32_t)v;
  const bool reached = depth[v] >= 0;
  if (reached && v != source) bc[c] += sigma[v] * acc[v];
  if (sigma_out) sigma_out[c] = reached ? sigma[v] : 0.0;
}

inline unsigned blocks_of(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_bc_levels(const int32_t* depth, const int32_t* R, int64_t V, int32_t source,
                            int32_t n_levels, uint32_t* lvl_n, unsigned long long* lvl_m,
                            double* sigma, double* acc, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  k_bc_level_count<<<blocks_of(V, (int64_t)kBcBlock * kBcItems), kBcBlock, 0, st>>>(
      depth, R, V, source, n_levels, lvl_n, lvl_m, sigma, acc);
  return hipGetLastError();
}

hipError_t launch_bc_scatter(const int32_t* depth, int64_t V, int32_t n_levels, uint32_t* cursor,
                             int32_t* levels, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  k_bc_level_scatter<<<blocks_of(V, (int64_t)kBcBlock * kBcItems), kBcBlock, 0, st>>>(
      depth, V, n_levels, cursor, levels);
  return hipGetLastError();
}

hipError_t launch_bc_sigma(int mode, const int32_t* frontier, const int32_t* offsets,
                           const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                           int64_t m_f, const int32_t* R, const int32_t* C, const int32_t* depth,
                           double* sigma, int32_t next_depth, const AdvCfg& cfg, hipStream_t st) {
  const BcSigma f{depth, sigma, next_depth};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st);
}

hipError_t launch_bc_dependency(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C,
                                const int32_t* depth, const double* sigma, double* acc,
                                int32_t prev_depth, const AdvCfg& cfg, hipStream_t st) {
  const BcDependency f{depth, sigma, acc, prev_depth};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st);
}

hipError_t launch_bc_finalize(const int32_t* depth, const double* sigma, const double* acc,
                              int64_t V, int32_t source, const int32_t* perm, double* bc,
                              double* sigma_out, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  k_bc_finalize<<<blocks_of(V, kBcBlock), kBcBlock, 0, st>>>(depth, sigma, acc, V, source, perm,
                                                             bc, sigma_out);
  return hipGetLastError();
}

}  // namespace gr
