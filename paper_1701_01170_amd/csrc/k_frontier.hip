// Frontier bookkeeping kernels: BFS initialisation (Alg. 1, Set_Problem_Data),
// frontier statistics and the degree prefix-sum that gives advance its scatter
// offsets (Sec. 4.1, the allocation stage), and small bitmap utilities.
#include "gr_internal.h"
#include "k_common.h"

namespace gr {

namespace {

constexpr int kStatsBlock = 256;
constexpr int kStatsGrid = 512;
// Frontier entries a thread handles per round.  Their loads (queue entry, then
// two row offsets) are all issued before any result is used, and past the
// slice end they read the slice's last entry instead of branching: a branch
// around each load would make every load wait for the one before it.
constexpr int kStatsItems = 8;

__global__ __launch_bounds__(256) void k_bfs_init(int32_t* __restrict__ depth,
                                                  int32_t* __restrict__ parent, int64_t V,
                                                  uint32_t* __restrict__ bm, int64_t n_words,
                                                  int32_t source, int32_t* __restrict__ queue,
                                                  Ctrl* __restrict__ ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t v = i0; v < V; v += stride) {
    depth[v] = (v == source) ? 0 : -1;
    if (parent) parent[v] = -1;
  }
  // level 0 has parity 0: old = even words (the source), live = odd words (empty)
  for (int64_t w = i0; w < n_words; w += stride) {
    bm[2 * w] = (w == (source >> 5)) ? (1u << (source & 31)) : 0u;
    bm[2 * w + 1] = 0u;
  }
  if (i0 == 0) {
    queue[0] = source;
    ctrl->q_count[0] = 1;
    ctrl->q_count[1] = 0;
    ctrl->q_count[2] = 0;
    ctrl->m_f[0] = ctrl->m_f[1] = 0;
    ctrl->max_deg[0] = ctrl->max_deg[1] = 0;
    ctrl->inspected = 0;
    ctrl->reached_edges = 0;
    ctrl->ul_count[0] = ctrl->ul_count[1] = 0;
  }
}

// Degree sum / max of the frontier, one contiguous slice per block.  Block
// sums go to block_sums[b] (the offsets kernel scans them); totals are
// accumulated atomically in slot `parity`, which the previous call cleared.
// Block 0 clears the other slot and the two counters the next step appends to.
__device__ __forceinline__ void frontier_stats(const int32_t* __restrict__ frontier, int64_t n_f,
                                               const int32_t* __restrict__ R,
                                               int64_t* __restrict__ block_sums,
                                               Ctrl* __restrict__ ctrl, int parity,
                                               uint32_t* zero_a, uint32_t* zero_b) {
  __shared__ int64_t s_sum[kStatsBlock / kWave];
  __shared__ int64_t s_max[kStatsBlock / kWave];
  const int G = gridDim.x;
  const int64_t per = (n_f + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n_f ? lo + per : n_f;
  int64_t sum = 0, mx = 0;
  for (int64_t base = lo; base < hi; base += (int64_t)kStatsBlock * kStatsItems) {
    int32_t u[kStatsItems], a[kStatsItems], b[kStatsItems];
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      const int64_t i = base + r * kStatsBlock + threadIdx.x;
      u[r] = frontier[i < hi ? i : hi - 1];
    }
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      a[r] = R[u[r]];
      b[r] = R[u[r] + 1];
    }
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      const int64_t d = base + r * kStatsBlock + threadIdx.x < hi ? (int64_t)b[r] - a[r] : 0;
      sum += d;
      mx = d > mx ? d : mx;
    }
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
    int64_t bs = 0, bmx = 0;
    for (int i = 0; i < kStatsBlock / kWave; ++i) {
      bs += s_sum[i];
      bmx = s_max[i] > bmx ? s_max[i] : bmx;
    }
    block_sums[blockIdx.x] = bs;
    if (bs) atomicAdd((unsigned long long*)&ctrl->m_f[parity], (unsigned long long)bs);
    if (bmx) atomicMax((unsigned long long*)&ctrl->max_deg[parity], (unsigned long long)bmx);
    if (blockIdx.x == 0) {
      ctrl->n_f[parity] = n_f;
      ctrl->m_f[parity ^ 1] = 0;
      ctrl->max_deg[parity ^ 1] = 0;
      if (zero_a) *zero_a = 0;
      if (zero_b) *zero_b = 0;
    }
  }
}

__global__ __launch_bounds__(kStatsBlock) void k_frontier_stats(
    const int32_t* __restrict__ frontier, const uint32_t* __restrict__ n_f_dev,
    const int32_t* __restrict__ R, int64_t* __restrict__ block_sums, Ctrl* __restrict__ ctrl,
    int parity, uint32_t* zero_a, uint32_t* zero_b) {
  frontier_stats(frontier, (int64_t)*n_f_dev, R, block_sums, ctrl, parity, zero_a, zero_b);
}

// The same for the frontier left by a block of device-predicated levels: the
// block ran ctrl->dl_levels of them, so its last frontier is queue
// (cur0 + dl_levels) % 3 and the next appends go to the queue after it.
__global__ __launch_bounds__(kStatsBlock) void k_frontier_stats_after_block(
    Queues3 qs, int cur0, const int32_t* __restrict__ R, int64_t* __restrict__ block_sums,
    Ctrl* __restrict__ ctrl, int parity) {
  const int cur = (cur0 + ctrl->dl_levels) % 3;
  frontier_stats(qs.q[cur], (int64_t)ctrl->q_count[cur], R, block_sums, ctrl, parity,
                 &ctrl->q_count[(cur + 1) % 3], nullptr);
}

// Exclusive scan of frontier degrees into offsets[0..n_f] (same slicing as
// k_frontier_stats; each block sums the block totals before it), the row
// start of every frontier vertex, and the chunk -> segment map of
// output-balanced LB: chunk_start[c] = the frontier index whose neighbour list
// holds edge c * chunk (the sorted search of 0, N, 2N, ... in the offsets).
__global__ __launch_bounds__(kStatsBlock) void k_frontier_offsets(
    const int32_t* __restrict__ frontier, int64_t n_f, const uint32_t* __restrict__ n_f_dev,
    const int32_t* __restrict__ R, const int64_t* __restrict__ block_sums,
    const int64_t* __restrict__ total, int32_t* __restrict__ offsets,
    int32_t* __restrict__ rstart, int32_t* __restrict__ chunk_start, int32_t chunk) {
  __shared__ int64_t s_tot[kStatsBlock / kWave + 1];
  if (n_f_dev) n_f = *n_f_dev;
  const int G = gridDim.x;
  const int64_t per = (n_f + G - 1) / G;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n_f ? lo + per : n_f;
  // prefix of the block sums before this block
  int64_t pre = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kStatsBlock) pre += block_sums[b];
  {
    int64_t t;
    block_excl_scan<kStatsBlock>(pre, s_tot, &t);
    pre = t;
  }
  // kStatsItems consecutive entries per thread and round
  int64_t run = pre;
  for (int64_t base = lo; base < hi; base += (int64_t)kStatsBlock * kStatsItems) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kStatsItems;
    int32_t u[kStatsItems], a[kStatsItems], b[kStatsItems];
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) u[r] = frontier[i0 + r < hi ? i0 + r : hi - 1];
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      a[r] = R[u[r]];
      b[r] = R[u[r] + 1];
    }
    int64_t d[kStatsItems], tsum = 0;
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      d[r] = i0 + r < hi ? (int64_t)b[r] - a[r] : 0;
      tsum += d[r];
    }
    int64_t tot;
    int64_t o = run + block_excl_scan<kStatsBlock>(tsum, s_tot, &tot);
#pragma unroll
    for (int r = 0; r < kStatsItems; ++r) {
      const int64_t i = i0 + r;
      if (i < hi) {
        offsets[i] = (int32_t)o;
        rstart[i] = a[r];
        for (int64_t c = (o + chunk - 1) / chunk; c * chunk < o + d[r]; ++c) chunk_start[c] = (int32_t)i;
      }
      o += d[r];
    }
    run += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[n_f] = (int32_t)*total;
}

// live |= old over all word pairs
__global__ __launch_bounds__(256) void k_bitmap_merge(uint32_t* __restrict__ bm, int p,
                                                      int64_t n_words) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < n_words) {
    uint2 x = reinterpret_cast<uint2*>(bm)[w];
    if (p == 0) x.y |= x.x;
    else x.x |= x.y;
    reinterpret_cast<uint2*>(bm)[w] = x;
  }
}

// out[c] = in[inv[c]] over the caller's ids c: the writes are coalesced and the
// random accesses are reads (scattering out[perm[i]] = in[i] took 67 us per
// R-MAT 22 BFS, twice as long).  kPermItems entries per thread, their loads
// issued before any is used.
constexpr int kPermItems = 4;
__global__ __launch_bounds__(256) void k_permute_out(const int32_t* __restrict__ inv, int64_t V,
                                                     const int32_t* __restrict__ depth_in,
                                                     const int32_t* __restrict__ parent_in,
                                                     int32_t* __restrict__ depth_out,
                                                     int32_t* __restrict__ parent_out) {
  const int64_t c0 = (int64_t)blockIdx.x * (256 * kPermItems) + threadIdx.x;
  int32_t v[kPermItems], d[kPermItems], pa[kPermItems];
#pragma unroll
  for (int r = 0; r < kPermItems; ++r) {
    const int64_t c = c0 + r * 256;
    v[r] = c < V ? inv[c] : 0;
  }
#pragma unroll
  for (int r = 0; r < kPermItems; ++r) {
    d[r] = depth_in[v[r]];
    pa[r] = parent_out ? parent_in[v[r]] : 0;
  }
#pragma unroll
  for (int r = 0; r < kPermItems; ++r) {
    const int64_t c = c0 + r * 256;
    if (c >= V) break;
    depth_out[c] = d[r];
    if (parent_out) parent_out[c] = pa[r];
  }
}

// Copy the control block to host memory: every thread orders its own stores
// at system scope before the workgroup barrier, then one thread releases the
// sequence number the host waits for.
__global__ __launch_bounds__(128) void k_publish(const uint32_t* __restrict__ src,
                                                 uint32_t* __restrict__ dst, int n_words,
                                                 uint32_t* flag, uint32_t seq, PublishExtra x) {
  for (int i = threadIdx.x; i < n_words; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < x.n_words; i += blockDim.x) x.dst[i] = x.src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n,
                                                  uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// Start of a device-predicated block whose first frontier is queue cur: the
// block counters, the visited counts before that frontier and the priority
// queue state of its first step.
__global__ void k_dl_begin(Ctrl* __restrict__ ctrl, int cur, int64_t vm, int64_t vn,
                           uint32_t pq_T, int32_t pq_epoch, int32_t pq_fc) {
  ctrl->dl_levels = 0;
  ctrl->dl_stop = 0;
  ctrl->q_count[(cur + 1) % 3] = 0;
  ctrl->dl_vm[0] = vm;
  ctrl->dl_vn[0] = vn;
  ctrl->pq_T[0] = pq_T;
  ctrl->pq_epoch[0] = pq_epoch;
  ctrl->pq_fc[0] = pq_fc;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int stats_grid() { return kStatsGrid; }

hipError_t launch_bfs_init(int32_t* depth, int32_t* parent, int64_t V, uint32_t* bm,
                           int64_t n_words, int32_t source, int32_t* queue, Ctrl* ctrl,
                           hipStream_t st) {
  const int64_t n = V > n_words ? V : n_words;
  unsigned g = blocks_for(n, 256);
  if (g > 4096) g = 4096;
  k_bfs_init<<<g, 256, 0, st>>>(depth, parent, V, bm, n_words, source, queue, ctrl);
  return hipGetLastError();
}

hipError_t launch_frontier_stats(const int32_t* frontier, const uint32_t* n_f_dev, const int32_t* R,
                                 int64_t* block_sums, Ctrl* ctrl, int parity, uint32_t* zero_a,
                                 uint32_t* zero_b, hipStream_t st) {
  k_frontier_stats<<<kStatsGrid, kStatsBlock, 0, st>>>(frontier, n_f_dev, R, block_sums, ctrl,
                                                       parity, zero_a, zero_b);
  return hipGetLastError();
}

hipError_t launch_frontier_stats_after_block(const Queues3& qs, int cur0, const int32_t* R,
                                             int64_t* block_sums, Ctrl* ctrl, int parity,
                                             hipStream_t st) {
  k_frontier_stats_after_block<<<kStatsGrid, kStatsBlock, 0, st>>>(qs, cur0, R, block_sums, ctrl,
                                                                   parity);
  return hipGetLastError();
}

hipError_t launch_frontier_offsets(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                   const int64_t* block_sums, const int64_t* total,
                                   int32_t* offsets, int32_t* rstart, int32_t* chunk_start,
                                   int32_t chunk, hipStream_t st, const uint32_t* n_f_dev) {
  k_frontier_offsets<<<kStatsGrid, kStatsBlock, 0, st>>>(frontier, n_f, n_f_dev, R, block_sums,
                                                         total, offsets, rstart, chunk_start,
                                                         chunk);
  return hipGetLastError();
}

hipError_t launch_bitmap_merge(uint32_t* bm, int p, int64_t n_words, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  k_bitmap_merge<<<blocks_for(n_words, 256), 256, 0, st>>>(bm, p, n_words);
  return hipGetLastError();
}

hipError_t launch_dl_begin(Ctrl* ctrl, int cur, int64_t vm, int64_t vn, uint32_t pq_T,
                           int32_t pq_epoch, int32_t pq_fc, hipStream_t st) {
  k_dl_begin<<<1, 1, 0, st>>>(ctrl, cur, vm, vn, pq_T, pq_epoch, pq_fc);
  return hipGetLastError();
}

hipError_t launch_permute_out(const int32_t* inv, int64_t V, const int32_t* depth_in,
                              const int32_t* parent_in, int32_t* depth_out, int32_t* parent_out,
                              hipStream_t st) {
  if (V <= 0) return hipSuccess;
  k_permute_out<<<blocks_for(V, 256 * kPermItems), 256, 0, st>>>(inv, V, depth_in, parent_in,
                                                                 depth_out, parent_out);
  return hipGetLastError();
}

hipError_t launch_publish(const Ctrl* src, Ctrl* host_dst, uint32_t* host_flag, uint32_t seq,
                          hipStream_t st, const PublishExtra& extra) {
  static_assert(sizeof(Ctrl) % 4 == 0, "control block is copied as 32-bit words");
  k_publish<<<1, 128, 0, st>>>(reinterpret_cast<const uint32_t*>(src),
                               reinterpret_cast<uint32_t*>(host_dst), (int)(sizeof(Ctrl) / 4),
                               host_flag, seq, extra);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_u32<<<blocks_for(n, 256), 256, 0, st>>>(p, n, value);
  return hipGetLastError();
}

}  // namespace gr
