// Frontier bookkeeping kernels: BFS initialisation (Alg. 1, Set_Problem_Data),
// frontier statistics and the degree prefix-sum that gives advance its scatter
// offsets (Sec. 4.1, the allocation stage), the unvisited-frontier generation
// of the pull traversal (Alg. 2), and small bitmap utilities.
#include "gr_internal.h"
#include "k_common.h"

namespace gr {

namespace {

constexpr int kStatsBlock = 256;
constexpr int kStatsGrid = 512;

__global__ __launch_bounds__(256) void k_bfs_init(int32_t* __restrict__ depth,
                                                  int32_t* __restrict__ parent, int64_t V,
                                                  uint32_t* __restrict__ bm_old,
                                                  uint32_t* __restrict__ bm_live, int64_t n_words,
                                                  int32_t source, int32_t* __restrict__ queue,
                                                  Ctrl* __restrict__ ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t v = i0; v < V; v += stride) {
    depth[v] = (v == source) ? 0 : -1;
    if (parent) parent[v] = -1;
  }
  for (int64_t w = i0; w < n_words; w += stride) {
    bm_old[w] = (w == (source >> 5)) ? (1u << (source & 31)) : 0u;
    bm_live[w] = 0u;
  }
  if (i0 == 0) {
    queue[0] = source;
    ctrl->q_count[0] = 1;
    ctrl->q_count[1] = 0;
    ctrl->u_count[0] = 0;
    ctrl->u_count[1] = 0;
    ctrl->inspected = 0;
    ctrl->reached_edges = 0;
    ctrl->misc[0] = 0;  // statistics ticket
  }
}

// Per-block degree sum / max over a contiguous slice of the frontier.  The
// last block to finish (ticket in ctrl->misc[0]) scans the block sums into
// exclusive block prefixes, publishes m_f / max degree / n_f in the control
// block and clears the two queue counters the next step will append to.
// block_sums layout: [0,G) sums, [G,2G) maxima, [2G,3G) exclusive prefixes,
// [3G] total.
__global__ __launch_bounds__(kStatsBlock) void k_frontier_stats(
    const int32_t* __restrict__ frontier, const uint32_t* __restrict__ n_f_dev,
    const int32_t* __restrict__ R, int64_t* __restrict__ block_sums, Ctrl* __restrict__ ctrl,
    uint32_t* zero_a, uint32_t* zero_b) {
  __shared__ int64_t s_sum[kStatsBlock / kWave];
  __shared__ int64_t s_max[kStatsBlock / kWave];
  __shared__ bool s_last;
  const int G = gridDim.x;
  const int64_t n_f = (int64_t)*n_f_dev;
  const int64_t per = (n_f + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n_f ? lo + per : n_f;
  int64_t sum = 0, mx = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kStatsBlock) {
    int32_t u = frontier[i];
    int64_t d = (int64_t)R[u + 1] - R[u];
    sum += d;
    mx = d > mx ? d : mx;
  }
  sum = wave_sum(sum);
  mx = wave_max(mx);
  const int w = threadIdx.x / kWave;
  if (lane() == 0) {
    s_sum[w] = sum;
    s_max[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t bs = 0, bm = 0;
    for (int i = 0; i < kStatsBlock / kWave; ++i) {
      bs += s_sum[i];
      bm = s_max[i] > bm ? s_max[i] : bm;
    }
    block_sums[blockIdx.x] = bs;
    block_sums[G + blockIdx.x] = bm;
    __threadfence();
    unsigned long long t = atomicAdd((unsigned long long*)&ctrl->misc[0], 1ull);
    s_last = (t == (unsigned long long)(G - 1));
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // last block: scan G block sums (G <= 64 * kStatsBlock / kWave * ... handled serially per thread)
  __shared__ int64_t s_tot[kStatsBlock / kWave + 1];
  int64_t run_base = 0, total_max = 0;
  for (int base = 0; base < G; base += kStatsBlock) {
    int b = base + threadIdx.x;
    int64_t x = b < G ? block_sums[b] : 0;
    int64_t m = b < G ? block_sums[G + b] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan<kStatsBlock>(x, s_tot, &tot);
    if (b < G) block_sums[2 * G + b] = run_base + ex;
    run_base += tot;
    m = wave_max(m);
    if (lane() == 0) s_max[w] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 0; i < kStatsBlock / kWave; ++i) total_max = s_max[i] > total_max ? s_max[i] : total_max;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    block_sums[3 * G] = run_base;
    ctrl->m_f = run_base;
    ctrl->max_deg = total_max;
    ctrl->n_f = n_f;
    ctrl->misc[0] = 0;
    if (zero_a) *zero_a = 0;
    if (zero_b) *zero_b = 0;
  }
}

// Exclusive scan of frontier degrees into offsets[0..n_f] using the block
// prefixes of k_frontier_stats (same slicing).  Also marks every frontier
// vertex in the live visited bitmap (push steps keep live = visited through
// the next level).
__global__ __launch_bounds__(kStatsBlock) void k_frontier_offsets(
    const int32_t* __restrict__ frontier, int64_t n_f, const int32_t* __restrict__ R,
    const int64_t* __restrict__ block_sums, int32_t* __restrict__ offsets,
    uint32_t* __restrict__ live_bm) {
  __shared__ int64_t s_tot[kStatsBlock / kWave + 1];
  const int G = gridDim.x;
  const int64_t per = (n_f + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n_f ? lo + per : n_f;
  int64_t run = block_sums[2 * G + blockIdx.x];
  for (int64_t base = lo; base < hi; base += kStatsBlock) {
    int64_t i = base + threadIdx.x;
    int64_t d = 0;
    if (i < hi) {
      int32_t u = frontier[i];
      d = (int64_t)R[u + 1] - R[u];
      if (live_bm) atomicOr(&live_bm[u >> 5], 1u << (u & 31));
    }
    int64_t tot;
    int64_t ex = block_excl_scan<kStatsBlock>(d, s_tot, &tot);
    if (i < hi) offsets[i] = (int32_t)(run + ex);
    run += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[n_f] = (int32_t)block_sums[3 * G];
}

// Alg. 2, GenerateUnvisitedFrontier: every vertex not yet visited.  Vertices of
// degree zero are left out: in a symmetric graph nothing can reach them.
__global__ __launch_bounds__(256) void k_gen_unvisited(const uint32_t* __restrict__ bm_old,
                                                       const int32_t* __restrict__ R, int64_t V,
                                                       int32_t* __restrict__ out,
                                                       uint32_t* __restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool keep = false;
  if (v < V) keep = !bm_test(bm_old, (int32_t)v) && R[v + 1] > R[v];
  uint32_t slot = wave_append(count, keep);
  if (keep) out[slot] = (int32_t)v;
}

__global__ __launch_bounds__(256) void k_bitmap_or(uint32_t* __restrict__ dst,
                                                   const uint32_t* __restrict__ src,
                                                   int64_t n_words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_words) dst[i] |= src[i];
}

__global__ __launch_bounds__(256) void k_reached_edges(const int32_t* __restrict__ depth,
                                                       const int32_t* __restrict__ R, int64_t V,
                                                       int64_t* __restrict__ out) {
  __shared__ int64_t s[256 / kWave];
  int64_t acc = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * blockDim.x)
    if (depth[v] >= 0) acc += (int64_t)R[v + 1] - R[v];
  acc = wave_sum(acc);
  if (lane() == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < 256 / kWave; ++i) t += s[i];
    atomicAdd((unsigned long long*)out, (unsigned long long)t);
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n,
                                                  uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_u32<<<blocks_for(n, 256), 256, 0, st>>>(p, n, value);
  return hipGetLastError();
}

int stats_grid() { return kStatsGrid; }

hipError_t launch_bfs_init(int32_t* depth, int32_t* parent, int64_t V, uint32_t* bm_old,
                           uint32_t* bm_live, int64_t n_words, int32_t source, int32_t* queue,
                           Ctrl* ctrl, hipStream_t st) {
  int64_t n = V > n_words ? V : n_words;
  unsigned g = blocks_for(n, 256);
  if (g > 4096) g = 4096;
  k_bfs_init<<<g, 256, 0, st>>>(depth, parent, V, bm_old, bm_live, n_words, source, queue, ctrl);
  return hipGetLastError();
}

hipError_t launch_frontier_stats(const int32_t* frontier, const uint32_t* n_f_dev, const int32_t* R,
                                 int64_t* block_sums, Ctrl* ctrl, uint32_t* zero_a,
                                 uint32_t* zero_b, hipStream_t st) {
  k_frontier_stats<<<kStatsGrid, kStatsBlock, 0, st>>>(frontier, n_f_dev, R, block_sums, ctrl,
                                                       zero_a, zero_b);
  return hipGetLastError();
}

hipError_t launch_frontier_offsets(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                   const int64_t* block_sums, int32_t* offsets,
                                   uint32_t* live_bm, hipStream_t st) {
  k_frontier_offsets<<<kStatsGrid, kStatsBlock, 0, st>>>(frontier, n_f, R, block_sums, offsets,
                                                         live_bm);
  return hipGetLastError();
}

hipError_t launch_gen_unvisited(const uint32_t* bm_old, const int32_t* R, int64_t V,
                                int32_t* out_list, uint32_t* out_count, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  k_gen_unvisited<<<blocks_for(V, 256), 256, 0, st>>>(bm_old, R, V, out_list, out_count);
  return hipGetLastError();
}

hipError_t launch_bitmap_or(uint32_t* dst, const uint32_t* src, int64_t n_words, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  k_bitmap_or<<<blocks_for(n_words, 256), 256, 0, st>>>(dst, src, n_words);
  return hipGetLastError();
}

hipError_t launch_reached_edges(const int32_t* depth, const int32_t* R, int64_t V, int64_t* out,
                                hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 2048) g = 2048;
  k_reached_edges<<<g, 256, 0, st>>>(depth, R, V, out);
  return hipGetLastError();
}

}  // namespace gr
