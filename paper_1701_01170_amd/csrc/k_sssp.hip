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
#include "k_advance.h"
#include "k_dloop.h"

namespace gr {

namespace {

struct SsspVisit {
  const uint32_t* __restrict__ W;
  unsigned long long* __restrict__ keys;
  int32_t* __restrict__ tags;
  int32_t next_tag;

  using pay_t = int32_t;
  __device__ __forceinline__ int32_t seg_payload(int32_t u) const {
    return (int32_t)(uint32_t)(keys[u] >> 32);
  }
  __device__ __forceinline__ uint32_t edge_value(int64_t e) const { return W[e]; }
  __device__ __forceinline__ bool probe(int32_t u, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    if (cand >= 0xffffffffull) return false;  // cannot be a shortest distance (range checked at entry)
    const unsigned long long nk = (cand << 32) | (uint32_t)u;
    return nk < keys[v];                       // keys only decrease: otherwise nothing to gain
  }
  __device__ __forceinline__ bool commit(int32_t u, int32_t du, int32_t v, uint32_t w) const {
    const uint64_t cand = (uint64_t)(uint32_t)du + (uint64_t)w;
    const unsigned long long nk = (cand << 32) | (uint32_t)u;
    const unsigned long long old = atomicMin(&keys[v], nk);
    if (cand >= (old >> 32)) return false;     // no distance improvement (at most a better pred)
    return atomicExch(&tags[v], next_tag) != next_tag;
  }
  __device__ __forceinline__ void frontier_vertex(int32_t) const {}
};

__global__ __launch_bounds__(256) void k_sssp_init(unsigned long long* __restrict__ keys,
                                                   int32_t* __restrict__ tags, int64_t V,
                                                   Ctrl* __restrict__ ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
    keys[v] = ~0ull;
    tags[v] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->q_count[1] = 0;
    ctrl->q_count[2] = 0;
    ctrl->u_count[0] = 0;
    ctrl->u_count[1] = 0;
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
                                                       int64_t* __restrict__ reached_edges) {
  __shared__ int64_t s[256 / kWave];
  int64_t acc = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V;
       v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[v];
    const uint32_t d = (uint32_t)(k >> 32);
    dist[v] = d;
    if (pred) pred[v] = (int32_t)(uint32_t)(k & 0xffffffffull);
    if (d != 0xffffffffu) acc += (int64_t)R[v + 1] - R[v];
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

hipError_t launch_sssp_init(unsigned long long* keys, int32_t* tags, int64_t V, Ctrl* ctrl,
                            hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 4096) g = 4096;
  k_sssp_init<<<g, 256, 0, st>>>(keys, tags, V, ctrl);
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
                             unsigned long long* keys, int32_t* tags, int32_t next_tag,
                             int32_t* out_q, uint32_t* out_count, int chunk, hipStream_t st) {
  SsspVisit f{W, keys, tags, next_tag};
  return push_dispatch(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R, C, f, out_q,
                       out_count, chunk, st);
}

hipError_t launch_sssp_finalize(const unsigned long long* keys, const int32_t* R, int64_t V,
                                uint32_t* dist, int32_t* pred, const int32_t* src_dev,
                                int32_t n_src, int64_t* reached_edges, hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 4096) g = 4096;
  k_sssp_finalize<<<g, 256, 0, st>>>(keys, R, V, dist, pred, reached_edges);
  if (pred) k_sssp_source_pred<<<blocks_for(n_src, 256), 256, 0, st>>>(src_dev, n_src, pred);
  return hipGetLastError();
}

hipError_t launch_sssp_dstep(const DlArgs& a, const uint32_t* W, unsigned long long* keys,
                             int32_t* tags, int32_t next_tag, int n_blocks, hipStream_t st) {
  const SsspVisit f{W, keys, tags, next_tag};
  k_dstep<SsspVisit><<<n_blocks, kAdvBlock, 0, st>>>(a, f);
  return hipGetLastError();
}

}  // namespace gr
