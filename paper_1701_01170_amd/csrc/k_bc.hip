// Betweenness centrality (Sec. 6, betweenness centrality; Brandes's two
// passes) on the advance operator.  The forward pass is the BFS (depths) and
// then, level by level, sigma(w) = sum of sigma(u) over the edges (u, w) from
// the level before; the backward pass walks the levels in reverse with
// acc(v) = sum over v's successors w (edges into the level after) of
// (1 + delta(w)) / sigma(w) = 1 / sigma(w) + acc(w), so that
// delta(v) = sigma(v) * acc(v).  Each sum over the edges between two adjacent
// levels is either pushed (the level the terms come from sweeps its rows and
// adds each term into the other end with a hardware fp64 atomic; device
// memory from hipMalloc, coarse grained) or pulled (the level the sums belong
// to sweeps its own rows and reduces them without per-edge atomics; the graph
// is symmetric, so a vertex's row holds its predecessors and successors).
// Both forms use the traversals' LB mapping; levels come from a counting sort
// of the depths, so every level's vertices are contiguous and one degree scan
// over them serves every level.
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

// Per-edge values summed by the pull passes: sigma(u) of a predecessor in the
// forward pass, (1 + delta(w)) / sigma(w) = 1 / sigma(w) + acc(w) of a
// successor in the backward pass.
struct BcSigmaVal {
  const double* __restrict__ sigma;
  __device__ __forceinline__ double operator()(int32_t u) const { return sigma[u]; }
};
struct BcDependencyVal {
  const double* __restrict__ sigma;
  const double* __restrict__ acc;
  __device__ __forceinline__ double operator()(int32_t w) const { return 1.0 / sigma[w] + acc[w]; }
};

// Sum over the 64 lanes' consecutive edges by segment (key non-decreasing
// over the lanes): each lane gets the sum of its key's lanes up to itself;
// *last marks the last lane of each key's run.
__device__ __forceinline__ double wave_seg_sum(double x, int key, bool* last) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(x, o);
    const int ky = __shfl_up(key, o);
    if (lane() >= o && ky == key) x += y;
  }
  const int kn = __shfl_down(key, 1);
  *last = lane() == kWave - 1 || kn != key;
  return x;
}

// Pull form of a pass (the vertex that owns a sum gathers it, instead of the
// sum being scattered onto it by atomics): for every vertex v of a level and
// every edge (v, w) with depth(w) == want, out(v) += val(w).  On a symmetric
// graph this is the push form's sum with the edge's ends swapped: the
// dependency of v gathers over its successors one level deeper, sigma(w) over
// its predecessors one level up.  Where a few vertices of the level before
// receive most of a large level's edges (hubs of a power-law graph) the push
// form queues every edge's fp64 atomic on those few addresses; here no edge
// makes an atomic.  The rows are balanced as in k_push_lb (equal chunks of the
// level's edges per workgroup, the chunk -> first-row map from the offsets
// kernel, each edge's row from a max-scan of row starts); every wavefront
// reduces its 64 consecutive edges by row with a shuffle scan, the last lane
// of each run adds the run into its row's LDS slot, and each row the chunk
// touches is written once: a plain store when the chunk holds the whole row
// (out starts at 0 and no other workgroup writes it), else one fp64 atomic.
template <class Val, int EPT, int NB>
__global__ __launch_bounds__(kBcBlock) void k_bc_pull_lb(
    const int32_t* __restrict__ frontier, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ rstart, const int32_t* __restrict__ chunk_start, int32_t n_f,
    int32_t m_f, int64_t e_base, const int32_t* __restrict__ C, const int32_t* __restrict__ depth,
    int32_t want, Val val, double* __restrict__ out) {
  constexpr int BATCH = kBcBlock * EPT;
  constexpr int N = BATCH * NB;
  constexpr int SPT = N / kBcBlock;
  constexpr int CAP = lb_cap(N);
  constexpr int kNoRow = 0xFFFF;  // lanes past the chunk's last edge (above every row index)
  __shared__ uint16_t s_seg[N];
  __shared__ int32_t s_off[CAP + 1];
  __shared__ int32_t s_u[CAP];
  __shared__ int32_t s_rb[CAP];
  __shared__ double s_sum[CAP];
  __shared__ int32_t s_tmp[kBcBlock / kWave + 1];
  const int c = blockIdx.x;
  const int64_t e0 = e_base + (int64_t)c * N;
  const int64_t e1 = e0 + N < e_base + m_f ? e0 + N : e_base + m_f;
  const int nchunks = (int)(((int64_t)m_f + N - 1) / N);
  const int sb = chunk_start[c];
  const int se = c + 1 < nchunks ? chunk_start[c + 1] : n_f - 1;
  for (int pb = sb; pb <= se; pb += CAP) {
    const int cnt = (se - pb + 1) < CAP ? (se - pb + 1) : CAP;
    for (int i = threadIdx.x; i < cnt; i += kBcBlock) {
      const int s = pb + i;
      s_off[i] = offsets[s];
      s_u[i] = frontier[s];
      s_rb[i] = rstart[s];
      s_sum[i] = 0.0;
    }
    if (threadIdx.x == 0) s_off[cnt] = offsets[pb + cnt];
    for (int j = threadIdx.x; j < N; j += kBcBlock) s_seg[j] = 0;
    __syncthreads();
    const int64_t lo = e0 > (int64_t)s_off[0] ? e0 : (int64_t)s_off[0];
    const int64_t hi = e1 < (int64_t)s_off[cnt] ? e1 : (int64_t)s_off[cnt];
    for (int k = 1 + threadIdx.x; k < cnt; k += kBcBlock) {
      const int64_t pos = (int64_t)s_off[k] - lo;
      if (pos < hi - lo && s_off[k + 1] > s_off[k]) s_seg[pos] = (uint16_t)k;
    }
    __syncthreads();
    lb_seg_maxscan<SPT, kBcBlock>(s_seg, s_tmp);
    __syncthreads();
    for (int b = 0; b < NB; ++b) {
      if (lo + (int64_t)b * BATCH >= hi) break;
      int key[EPT];
      int32_t w[EPT];
      double x[EPT];
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        const int j = b * BATCH + r * kBcBlock + threadIdx.x;
        const int64_t e = lo + j;
        key[r] = e < hi ? (int)s_seg[j] : kNoRow;
        w[r] = key[r] != kNoRow ? C[s_rb[key[r]] + (int32_t)(e - s_off[key[r]])] : 0;
      }
#pragma unroll
      for (int r = 0; r < EPT; ++r)
        if (key[r] != kNoRow && depth[w[r]] != want) w[r] = -1;
#pragma unroll
      for (int r = 0; r < EPT; ++r) x[r] = key[r] != kNoRow && w[r] >= 0 ? val(w[r]) : 0.0;
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        bool last;
        const double sum = wave_seg_sum(x[r], key[r], &last);
        if (last && key[r] != kNoRow && sum != 0.0) atomicAdd(&s_sum[key[r]], sum);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kBcBlock) {
      const int64_t a = s_off[i], z = s_off[i + 1];
      if (z <= lo || a >= hi || z <= a) continue;  // no edge of this row in the chunk
      if (a >= e0 && z <= e1)
        out[s_u[i]] = s_sum[i];
      else if (s_sum[i] != 0.0)
        unsafeAtomicAdd(&out[s_u[i]], s_sum[i]);
    }
    __syncthreads();
  }
}

// The chunk -> first-row maps of the pull passes for every level in one
// launch.  The n_r reached vertices are stored level after level (`levels`)
// and `offsets` is one exclusive scan of their degrees over all of them, so
// level x's rows are vertex indexes tab[x] .. and its edges positions
// tab[L + x] ..; its chunks of `chunk` edges, counted from its first edge, are
// entries tab[2L + x] .. of chunk_map, each set to the level-local index of
// the row holding the chunk's first edge (the sorted search of 0, N, 2N, ...
// done by scattering from the rows).
__global__ __launch_bounds__(kBcBlock) void k_bc_chunk_map(
    const int32_t* __restrict__ levels, const int32_t* __restrict__ depth, int64_t n_r,
    const int32_t* __restrict__ offsets, const int64_t* __restrict__ tab, int32_t L,
    int32_t chunk, int32_t* __restrict__ chunk_map) {
  const int64_t i = (int64_t)blockIdx.x * kBcBlock + threadIdx.x;
  if (i >= n_r) return;
  const int32_t x = depth[levels[i]];
  const int64_t o = (int64_t)offsets[i] - tab[L + x];
  const int64_t d = (int64_t)offsets[i + 1] - offsets[i];
  int32_t* map = chunk_map + tab[2 * L + x];
  for (int64_t c = (o + chunk - 1) / chunk; c * chunk < o + d; ++c) map[c] = (int32_t)(i - tab[x]);
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
                           int64_t m_f, int64_t e_base, const int32_t* R, const int32_t* C,
                           const int32_t* depth, double* sigma, int32_t next_depth,
                           const AdvCfg& cfg, hipStream_t st) {
  const BcSigma f{depth, sigma, next_depth};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st, e_base);
}

hipError_t launch_bc_dependency(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, int64_t e_base, const int32_t* R, const int32_t* C,
                                const int32_t* depth, const double* sigma, double* acc,
                                int32_t prev_depth, const AdvCfg& cfg, hipStream_t st) {
  const BcDependency f{depth, sigma, acc, prev_depth};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, nullptr,
                       nullptr, cfg, st, e_base);
}

hipError_t launch_bc_chunk_map(const int32_t* levels, const int32_t* depth, int64_t n_r,
                               const int32_t* offsets, const int64_t* tab, int32_t n_levels,
                               int32_t chunk, int32_t* chunk_map, hipStream_t st) {
  if (n_r <= 0) return hipSuccess;
  k_bc_chunk_map<<<blocks_of(n_r, kBcBlock), kBcBlock, 0, st>>>(levels, depth, n_r, offsets, tab,
                                                                n_levels, chunk, chunk_map);
  return hipGetLastError();
}

hipError_t launch_bc_pull(bool dependency, const int32_t* frontier, const int32_t* offsets,
                          const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                          int64_t m_f, int64_t e_base, int chunk, const int32_t* C,
                          const int32_t* depth, int32_t want, double* sigma, double* acc,
                          hipStream_t st) {
  if (n_f <= 0 || m_f <= 0) return hipSuccess;
  const unsigned g = blocks_of(m_f, chunk);
#define GR_BC_PULL(CH)                                                                          \
  case CH: {                                                                                    \
    constexpr int ept = (CH / kBcBlock) < 16 ? (CH / kBcBlock) : 16;                            \
    constexpr int nb = CH / (kBcBlock * ept);                                                   \
    if (dependency)                                                                             \
      k_bc_pull_lb<BcDependencyVal, ept, nb><<<g, kBcBlock, 0, st>>>(                           \
          frontier, offsets, rstart, chunk_start, (int32_t)n_f, (int32_t)m_f, e_base, C, depth, \
          want, BcDependencyVal{sigma, acc}, acc);                                              \
    else                                                                                        \
      k_bc_pull_lb<BcSigmaVal, ept, nb><<<g, kBcBlock, 0, st>>>(                                \
          frontier, offsets, rstart, chunk_start, (int32_t)n_f, (int32_t)m_f, e_base, C, depth, \
          want, BcSigmaVal{sigma}, sigma);                                                      \
    break;                                                                                      \
  }
  switch (chunk) {
    GR_BC_PULL(512)
    GR_BC_PULL(1024)
    GR_BC_PULL(2048)
    GR_BC_PULL(4096)
    GR_BC_PULL(16384)
    default:
      GR_BC_PULL(8192)
  }
#undef GR_BC_PULL
  return hipGetLastError();
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
