// Multi-source BFS: up to 64 traversals share every sweep over the graph (the
// paper's future-work "higher-level task parallelism", Sec. 8: several BFS at
// once).  Per vertex, 64-bit masks hold one bit per source: `visit` (reached),
// `front` (in the current frontier of that source) and `next` (reached at this
// level).  One level:
//   expand   push: every active vertex u ORs front[u] & ~visit[v] into next[v]
//                  (atomic OR; the first setter appends v to the touched list);
//            pull: every vertex with unreached bits ORs front[u] over its
//                  neighbours (early exit once all its unreached bits appear);
//   finalize for every touched v: visit |= next, front' = next, and for each
//            new source bit s, depth[s][v] = d + 1 and parent[s][v] = the first
//            neighbour u (ascending) with bit s in front[u] = the smallest-id
//            parent of the single-source definition.
#include "k_advance.h"
#include "k_dloop.h"

namespace gr {

namespace {

using u64 = unsigned long long;

struct MsPush {
  const u64* __restrict__ visit;
  u64* __restrict__ next;
  using pay_t = u64;
  static constexpr bool kFar = false;
  static constexpr bool kBatchCommit = false;

  const u64* __restrict__ front;
  __device__ __forceinline__ u64 seg_payload(int32_t u) const { return front[u]; }
  __device__ __forceinline__ uint32_t edge_value(int64_t) const { return 0u; }
  __device__ __forceinline__ bool probe(int32_t, u64 fm, int32_t v, uint32_t) const {
    return (fm & ~visit[v]) != 0ull;
  }
  __device__ __forceinline__ bool commit(int32_t, u64 fm, int32_t v, uint32_t) const {
    const u64 m = fm & ~visit[v];
    return atomicOr(&next[v], m) == 0ull;  // first setter lists v once
  }
  // hooks of a device-predicated level (k_dstep): nothing to prepare or carry
  __device__ __forceinline__ void frontier_vertex(int32_t) const {}
  __device__ __forceinline__ MsPush prepare(const Ctrl*, int) const { return *this; }
  __device__ __forceinline__ void advance(Ctrl*, int, bool) const {}
};

__device__ __forceinline__ u64 wave_or(u64 x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x |= __shfl_xor(x, o);
  return x;
}

// Pull expansion over all vertices: lane per vertex for short lists, whole
// wavefront for long ones.  The scan is ascending with an early exit once all
// unreached bits appear, so the neighbour where a bit first appears is that
// source's smallest-id parent; with `parent` it is written here and the
// finalize pass skips its own parent search for this level.
__global__ __launch_bounds__(256) void k_ms_pull(int64_t V, const int32_t* __restrict__ R,
                                                 const int32_t* __restrict__ C,
                                                 const u64* __restrict__ front,
                                                 const u64* __restrict__ visit, u64 full,
                                                 u64* __restrict__ next, int32_t* __restrict__ touched,
                                                 uint32_t* __restrict__ n_touched,
                                                 int32_t* __restrict__ parent,
                                                 const int32_t* __restrict__ perm) {
  constexpr int U = 8;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < V;
  u64 need = 0;
  int32_t rb = 0, re = 0;
  int64_t vo = 0;  // v's caller id: the output column
  if (valid) {
    need = full & ~visit[v];
    if (need) {
      rb = R[v];
      re = R[v + 1];
      vo = perm ? perm[v] : v;
    }
  }
  u64 acc = 0;
  if (need && re - rb <= 64) {
    for (int32_t j0 = rb; j0 < re && (acc & need) != need; j0 += U) {
      int32_t u[U];
      u64 f[U];
#pragma unroll
      for (int r = 0; r < U; ++r) u[r] = j0 + r < re ? C[j0 + r] : -1;
#pragma unroll
      for (int r = 0; r < U; ++r) f[r] = u[r] >= 0 ? front[u[r]] : 0ull;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        u64 g = f[r] & need & ~acc;
        acc |= f[r];
        if (parent && g) {
          const int32_t uo = perm ? perm[u[r]] : u[r];
          for (; g; g &= g - 1) parent[(int64_t)(__ffsll(g) - 1) * V + vo] = uo;
        }
      }
    }
  }
  uint64_t big = __ballot(need != 0 && re - rb > 64);
  while (big) {
    const int l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const int32_t vb = __shfl(rb, l), ve = __shfl(re, l);
    const int64_t vv = __shfl(vo, l);
    const u64 nd = __shfl(need, l);
    u64 fnd = 0;  // bits of nd found so far
    for (int32_t base = vb; base < ve && fnd != nd; base += U * kWave) {
      int32_t u[U];
      u64 f[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int32_t j = base + r * kWave + lane();
        u[r] = j < ve ? C[j] : -1;
      }
#pragma unroll
      for (int r = 0; r < U; ++r) f[r] = u[r] >= 0 ? (front[u[r]] & nd) : 0ull;
      // ascending neighbour order inside the step: r-major, then lane
#pragma unroll
      for (int r = 0; r < U; ++r) {
        u64 g = wave_or(f[r]) & ~fnd;
        fnd |= g;
        if (parent) {
          while (g) {
            const int sb = __ffsll(g) - 1;
            g &= g - 1;
            const uint64_t b = __ballot((f[r] >> sb) & 1ull);
            const int32_t pu = __shfl(u[r], __ffsll((unsigned long long)b) - 1);
            if (lane() == 0) parent[(int64_t)sb * V + vv] = perm ? perm[pu] : pu;
          }
        }
      }
    }
    if (lane() == l) acc = fnd;
  }
  const u64 m = acc & need;
  if (m) next[v] = m;
  const uint32_t slot = wave_append(n_touched, m != 0ull);
  if (m) touched[slot] = (int32_t)v;
}

// Finalise the touched vertices: masks, depths, and (when the expansion did
// not find them) parents.
__global__ __launch_bounds__(256) void k_ms_finalize(
    const int32_t* __restrict__ touched, const uint32_t* __restrict__ n_touched,
    const int32_t* __restrict__ R, const int32_t* __restrict__ C, const u64* __restrict__ front,
    u64* __restrict__ front_next, u64* __restrict__ visit, u64* __restrict__ next,
    int32_t* __restrict__ depth, int32_t* __restrict__ parent, const int32_t* __restrict__ perm,
    int64_t V, int32_t next_depth, Ctrl* __restrict__ ctrl, bool predicated) {
  constexpr int U = 8;
  __shared__ int64_t s_pairs[256 / kWave], s_pe[256 / kWave];
  if (predicated && ctrl->dl_stop) return;  // a level of the block declined
  const int64_t n = *n_touched;
  if ((int64_t)blockIdx.x * blockDim.x >= n) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  int32_t v = 0, rb = 0, re = 0;
  int64_t vo = 0;  // v's caller id: the output column
  u64 nw = 0;
  if (valid) {
    v = touched[i];
    vo = perm ? perm[v] : v;
    nw = next[v];
    next[v] = 0;
    visit[v] |= nw;
    front_next[v] = nw;
    for (u64 b = nw; b; b &= b - 1) depth[(int64_t)(__ffsll(b) - 1) * V + vo] = next_depth;
    rb = R[v];
    re = R[v + 1];
  }
  // the pairs reached at this level and their degrees (selector features)
  {
    const int64_t pc = __popcll(nw);
    const int64_t wp = wave_sum(pc), we = wave_sum(pc * (int64_t)(re - rb));
    if (lane() == 0) {
      s_pairs[threadIdx.x / kWave] = wp;
      s_pe[threadIdx.x / kWave] = we;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tp = 0, te = 0;
      for (int k = 0; k < 256 / kWave; ++k) {
        tp += s_pairs[k];
        te += s_pe[k];
      }
      if (tp) atomicAdd((unsigned long long*)&ctrl->ms_pairs, (unsigned long long)tp);
      if (te) atomicAdd((unsigned long long*)&ctrl->ms_pair_edges, (unsigned long long)te);
    }
  }
  if (!parent) return;
  // parents: first neighbour (ascending) carrying each new bit in its frontier mask
  u64 found = 0;
  if (valid && re - rb <= 256) {
    for (int32_t j0 = rb; j0 < re && found != nw; j0 += U) {
      int32_t u[U];
      u64 f[U];
#pragma unroll
      for (int r = 0; r < U; ++r) u[r] = j0 + r < re ? C[j0 + r] : -1;
#pragma unroll
      for (int r = 0; r < U; ++r) f[r] = u[r] >= 0 ? front[u[r]] : 0ull;
#pragma unroll
      for (int r = 0; r < U; ++r) {
        u64 g = f[r] & nw & ~found;
        found |= g;
        const int32_t uo = g ? (perm ? perm[u[r]] : u[r]) : 0;
        for (; g; g &= g - 1) parent[(int64_t)(__ffsll(g) - 1) * V + vo] = uo;
      }
    }
  }
  uint64_t big = __ballot(valid && re - rb > 256);
  while (big) {
    const int l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const int32_t vb = __shfl(rb, l), ve = __shfl(re, l);
    const int64_t vv = __shfl(vo, l);
    const u64 nd = __shfl(nw, l);
    u64 fnd = 0;
    for (int32_t base = vb; base < ve && fnd != nd; base += U * kWave) {
      int32_t u[U];
      u64 f[U];
#pragma unroll
      for (int r = 0; r < U; ++r) {
        const int32_t j = base + r * kWave + lane();
        u[r] = j < ve ? C[j] : -1;
      }
#pragma unroll
      for (int r = 0; r < U; ++r) f[r] = u[r] >= 0 ? (front[u[r]] & nd) : 0ull;
      // neighbour order inside the step: r-major, then lane
#pragma unroll
      for (int r = 0; r < U; ++r) {
        u64 g = wave_or(f[r]) & ~fnd;
        while (g) {
          const int s = __ffsll(g) - 1;
          g &= g - 1;
          const uint64_t b = __ballot((f[r] >> s) & 1ull);
          const int32_t pu = __shfl(u[r], __ffsll((unsigned long long)b) - 1);
          if (lane() == 0) parent[(int64_t)s * V + vv] = perm ? perm[pu] : pu;
          fnd |= 1ull << s;
        }
      }
    }
  }
}

// Sources: their bits in visit / front, depth 0, and the reached-pair
// counters start at the k source pairs.
__global__ __launch_bounds__(256) void k_ms_seed(const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ src_orig, int32_t k,
                                                 u64* __restrict__ visit, u64* __restrict__ front,
                                                 int32_t* __restrict__ depth, int64_t V,
                                                 const int32_t* __restrict__ R,
                                                 Ctrl* __restrict__ ctrl) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < k) {
    const int32_t v = src[s];
    atomicOr(&visit[v], 1ull << s);
    atomicOr(&front[v], 1ull << s);
    depth[(int64_t)s * V + src_orig[s]] = 0;
    atomicAdd((unsigned long long*)&ctrl->ms_pair_edges, (unsigned long long)(R[v + 1] - R[v]));
  }
  if (s == 0) atomicAdd((unsigned long long*)&ctrl->ms_pairs, (unsigned long long)k);
}

__global__ __launch_bounds__(256) void k_ms_clear(const int32_t* __restrict__ list,
                                                  const uint32_t* __restrict__ n,
                                                  u64* __restrict__ front,
                                                  const Ctrl* __restrict__ ctrl) {
  if (ctrl && ctrl->dl_stop) return;  // predicated: a level of the block declined
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)*n) front[list[i]] = 0ull;
}

// sum over v of popcount(visit[v]) * degree(v)
__global__ __launch_bounds__(256) void k_ms_teps(const u64* __restrict__ visit,
                                                 const int32_t* __restrict__ R, int64_t V,
                                                 int64_t* __restrict__ out) {
  __shared__ int64_t s[256 / kWave];
  // four vertices per thread and round, all loaded before any is used
  constexpr int K = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t acc = 0;
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < V; v0 += stride * K) {
    u64 m[K];
    int32_t a[K], b[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const int64_t v = v0 + r * stride < V ? v0 + r * stride : V - 1;
      m[r] = visit[v];
      a[r] = R[v];
      b[r] = R[v + 1];
    }
#pragma unroll
    for (int r = 0; r < K; ++r)
      if (v0 + r * stride < V) acc += (int64_t)__popcll(m[r]) * ((int64_t)b[r] - a[r]);
  }
  acc = wave_sum(acc);
  if (lane() == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < 256 / kWave; ++i) t += s[i];
    atomicAdd((unsigned long long*)out, (unsigned long long)t);
  }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_ms_seed(const int32_t* src_dev, const int32_t* src_orig_dev, int32_t k,
                          u64* visit, u64* front, int32_t* depth, int64_t V, const int32_t* R,
                          Ctrl* ctrl, hipStream_t st) {
  k_ms_seed<<<1, 256, 0, st>>>(src_dev, src_orig_dev, k, visit, front, depth, V, R, ctrl);
  return hipGetLastError();
}

hipError_t launch_ms_push(int mode, const int32_t* active, const int32_t* offsets,
                          const int32_t* rstart, const int32_t* chunk_start, int64_t n_a,
                          int64_t m_a, const int32_t* R, const int32_t* C, const u64* front,
                          const u64* visit, u64* next, int32_t* touched, uint32_t* n_touched,
                          const AdvCfg& cfg, hipStream_t st) {
  MsPush f{visit, next, front};
  return push_dispatch(mode, active, offsets, rstart, chunk_start, n_a, m_a, R, C, f, touched,
                       n_touched, cfg, st);
}

hipError_t launch_ms_pull(int64_t V, const int32_t* R, const int32_t* C, const u64* front,
                          const u64* visit, u64 full, u64* next, int32_t* touched,
                          uint32_t* n_touched, int32_t* parent, const int32_t* perm,
                          hipStream_t st) {
  k_ms_pull<<<blocks_for(V, 256), 256, 0, st>>>(V, R, C, front, visit, full, next, touched,
                                                n_touched, parent, perm);
  return hipGetLastError();
}

hipError_t launch_ms_finalize(const int32_t* touched, const uint32_t* n_touched, int64_t max_n,
                              const int32_t* R, const int32_t* C, const u64* front,
                              u64* front_next, u64* visit, u64* next, int32_t* depth,
                              int32_t* parent, const int32_t* perm, int64_t V, int32_t next_depth,
                              Ctrl* ctrl, hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  k_ms_finalize<<<blocks_for(max_n, 256), 256, 0, st>>>(touched, n_touched, R, C, front,
                                                        front_next, visit, next, depth, parent,
                                                        perm, V, next_depth, ctrl, false);
  return hipGetLastError();
}

hipError_t launch_ms_dlevel(const DlArgs& a, const MsLevel& m, int n_blocks, int64_t max_touched,
                            hipStream_t st) {
  const MsPush f{m.visit, m.next, m.front_cur};
  k_dstep<MsPush><<<n_blocks, kAdvBlock, 0, st>>>(a, f);
  const int next = (a.cur + 1) % 3;
  uint32_t* n_next = &a.ctrl->q_count[next];
  uint32_t* n_cur = &a.ctrl->q_count[a.cur];
  if (max_touched > 0)
    k_ms_finalize<<<blocks_for(max_touched, 256), 256, 0, st>>>(
        a.q_next, n_next, m.R, m.C, m.front_cur, m.front_next, m.visit, m.next, m.depth, m.parent,
        m.perm, m.V, m.next_depth, a.ctrl, true);
  k_ms_clear<<<blocks_for(a.max_n, 256), 256, 0, st>>>(a.q_cur, n_cur,
                                                      const_cast<u64*>(m.front_cur), a.ctrl);
  return hipGetLastError();
}

hipError_t launch_ms_clear(const int32_t* list, const uint32_t* n, int64_t max_n, u64* front,
                           hipStream_t st) {
  if (max_n <= 0) return hipSuccess;
  k_ms_clear<<<blocks_for(max_n, 256), 256, 0, st>>>(list, n, front, nullptr);
  return hipGetLastError();
}

hipError_t launch_ms_teps(const u64* visit, const int32_t* R, int64_t V, int64_t* out,
                          hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 1024) g = 1024;  // one atomic per workgroup, all on one address
  k_ms_teps<<<g, 256, 0, st>>>(visit, R, V, out);
  return hipGetLastError();
}

}  // namespace gr
