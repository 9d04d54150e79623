// Batched shortest paths: up to 16 single-source SSSP runs share each sweep
// over the graph (the paper's future-work task parallelism, Sec. 8, applied to
// Alg. 1).  Every vertex holds KS packed keys (dist << 32 | pred, one per
// source, as in the single-source relaxation) in one 8 * KS byte row, so the
// keys of a target vertex for all sources sit in one or two cache lines.  The
// frontier is the union of the sources' frontiers; amask[v] says for which
// sources v is active (its distance dropped in the previous iteration).
//
// One iteration:
//   relax  output-balanced like LB: each workgroup takes a chunk of the
//          frontier's edges and enumerates its (edge, active source) pairs,
//          consecutive lanes taking the sources of one edge (so their key
//          gathers share the target's row); a lane relaxes its pair with a
//          plain read of the target's key and a no-return atomic minimum
//          (Update_Label), and a lane that lowered the distance ORs its bit
//          into nmask[v]; the first setter appends v to the next frontier
//          (Remove_Redundant for the union);
//   clear  amask of the current frontier = 0;
//   move   for the next frontier: amask = nmask, nmask = 0, listing the
//          vertices with an active source left.
// With `relaxed` (nullable, KS words per vertex like the keys), each chunk
// raises relaxed[u][s] to 1 + the distance of (u, s) as it stages u, for every
// active source s of u (its items read the key after that, so they see that
// distance or a smaller one), and move resets it when the pair joins the next
// frontier.  A pair whose relaxed value equals 1 + its distance at move time
// was active and had every edge relaxed with that final distance, so move
// drops it (the single-source cull of vertices already relaxed with their
// final distance, per source); a value from an earlier iteration is larger
// than 1 + a distance that has dropped since, and 0 never matches.
// Keys only decrease, so a source's bit is set exactly when the vertex's
// distance for that source dropped in the iteration; every vertex then
// relaxes its edges with its final distance for every source at least once,
// and the key ends as the smallest (distance, predecessor) pair: the same
// canonical result as the single-source runs.
//
// Optional near / far split (Sec. 5.1 priority queue; one threshold T for all
// sources): an improvement to a distance >= T sets the pair's bit in fmask[v]
// instead of nmask[v] (the first setter puts v on the far pile).  When the
// frontier runs dry, T grows by delta and the far pile is split: pairs now
// below T join the frontier, pairs still above stay, pairs whose distance fell
// below the old threshold meanwhile were expanded with it already and are
// dropped.  Results are unchanged.
#include "k_advance.h"

namespace gr {

namespace {

using u64 = unsigned long long;

// Index of the r-th set bit (r < popcount) of a 16-bit mask.
__device__ __forceinline__ int select_bit(uint32_t m, int r) {
  int pos = 0;
#pragma unroll
  for (int w = 8; w > 0; w >>= 1) {
    const uint32_t lowm = m & ((1u << w) - 1u);
    const int c = __popc(lowm);
    if (r >= c) {
      r -= c;
      m >>= w;
      pos += w;
    } else {
      m = lowm;
    }
  }
  return pos;
}

template <int N, bool PQ>
__global__ __launch_bounds__(256) void k_msssp_relax(
    const int32_t* __restrict__ frontier, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ rstart, const int32_t* __restrict__ chunk_start, int32_t n_f,
    int32_t m_f, const int32_t* __restrict__ C, const uint32_t* __restrict__ W, int KS,
    u64* __restrict__ keys, const uint32_t* __restrict__ amask, uint32_t* __restrict__ nmask,
    uint32_t* __restrict__ fmask, int32_t* __restrict__ far_q, uint32_t* __restrict__ far_count,
    uint32_t T, const int32_t* __restrict__ perm, uint32_t* __restrict__ relaxed,
    int32_t* __restrict__ out_q, uint32_t* __restrict__ out_count) {
  constexpr int BLOCK = 256;
  constexpr int CAP = lb_cap(N);
  constexpr int SPT = (CAP + BLOCK - 1) / BLOCK;  // segments per thread in the item scan
  constexpr int B = 4;                            // items in flight per lane
  __shared__ int32_t s_off[CAP + 1];
  __shared__ int32_t s_u[CAP];
  __shared__ int32_t s_rb[CAP];
  __shared__ uint32_t s_am[CAP];
  __shared__ int32_t s_ioff[CAP + 1];  // first (edge, source) item of each segment in the chunk
  __shared__ int32_t s_tmp[BLOCK / kWave + 1];
  const int c = blockIdx.x;
  const int64_t e0 = (int64_t)c * N;
  const int64_t e1 = e0 + N < m_f ? e0 + N : m_f;
  const int nchunks = (int)(((int64_t)m_f + N - 1) / N);
  const int sb = chunk_start[c];
  const int se = c + 1 < nchunks ? chunk_start[c + 1] : n_f - 1;
  for (int pb = sb; pb <= se; pb += CAP) {
    const int cnt = (se - pb + 1) < CAP ? (se - pb + 1) : CAP;
    for (int i = threadIdx.x; i < cnt; i += BLOCK) {
      const int s = pb + i;
      const int32_t u = frontier[s];
      s_off[i] = offsets[s];
      s_u[i] = u;
      s_rb[i] = rstart[s];
      const uint32_t am = amask[u];
      s_am[i] = am;
      if (relaxed) {
        for (uint32_t b = am; b; b &= b - 1) {
          const int64_t x = (int64_t)u * KS + (__ffs(b) - 1);
          atomicMax(&relaxed[x], (uint32_t)(keys[x] >> 32) + 1u);
        }
      }
    }
    if (threadIdx.x == 0) s_off[cnt] = offsets[pb + cnt];
    __syncthreads();
    // items per segment = (its edges inside [e0, e1)) * (its active sources);
    // exclusive scan over the segments, SPT consecutive ones per thread
    int32_t part[SPT];
    int32_t run = 0;
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
      const int k = threadIdx.x * SPT + r;
      int32_t items = 0;
      if (k < cnt) {
        const int64_t a = s_off[k] > e0 ? s_off[k] : e0;
        const int64_t b = s_off[k + 1] < e1 ? s_off[k + 1] : e1;
        items = b > a ? (int32_t)(b - a) * __popc(s_am[k]) : 0;
      }
      part[r] = run;
      run += items;
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(run, s_tmp, &total);
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
      const int k = threadIdx.x * SPT + r;
      if (k < cnt) s_ioff[k] = ex + part[r];
    }
    if (threadIdx.x == 0) s_ioff[cnt] = total;
    __syncthreads();
    for (int32_t t0 = 0; t0 < total; t0 += BLOCK * B) {
      bool ok[B];
      int32_t u[B], ce[B], src[B], v[B];
      uint32_t w[B];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const int32_t t = t0 + r * BLOCK + threadIdx.x;
        ok[r] = t < total;
        int k = 0, sI = 0;
        int32_t e = 0;
        if (ok[r]) {
          k = upper_index(s_ioff, 0, cnt - 1, t);
          const uint32_t am = s_am[k];
          const int p = __popc(am);
          const int32_t j = t - s_ioff[k];
          const int32_t a = s_off[k] > e0 ? s_off[k] : (int32_t)e0;
          e = a + j / p;
          sI = select_bit(am, j % p);
        }
        u[r] = s_u[k];
        src[r] = sI;
        ce[r] = s_rb[k] + (e - s_off[k]);
      }
#pragma unroll
      for (int r = 0; r < B; ++r) {
        v[r] = ok[r] ? C[ce[r]] : 0;
        w[r] = ok[r] ? W[ce[r]] : 0u;
      }
      u64 ku[B], kv[B];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        ku[r] = ok[r] ? keys[(int64_t)u[r] * KS + src[r]] : 0ull;
        kv[r] = ok[r] ? keys[(int64_t)v[r] * KS + src[r]] : 0ull;
      }
      bool first[B], ffirst[B];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const uint64_t cand = (ku[r] >> 32) + (uint64_t)w[r];
        first[r] = ffirst[r] = false;
        if (ok[r] && cand < 0xffffffffull) {
          const u64 nk = (cand << 32) | (uint32_t)(perm ? perm[u[r]] : u[r]);
          if (nk < kv[r]) atomicMin(&keys[(int64_t)v[r] * KS + src[r]], nk);
          if (cand < (kv[r] >> 32)) {
            const uint32_t bit = 1u << src[r];
            if (!PQ || cand < (uint64_t)T) first[r] = atomicOr(&nmask[v[r]], bit) == 0u;
            else ffirst[r] = atomicOr(&fmask[v[r]], bit) == 0u;
          }
        }
      }
      uint32_t n_app = 0, n_far = 0;
#pragma unroll
      for (int r = 0; r < B; ++r) {
        n_app += first[r] ? 1u : 0u;
        n_far += ffirst[r] ? 1u : 0u;
      }
      if (__ballot(n_app != 0)) {
        const uint32_t inc = wave_incl_scan(n_app);
        uint32_t base = 0;
        if (lane() == kWave - 1) base = atomicAdd(out_count, inc);
        base = __shfl(base, kWave - 1) + inc - n_app;
#pragma unroll
        for (int r = 0; r < B; ++r)
          if (first[r]) out_q[base++] = v[r];
      }
      if constexpr (PQ) {
        if (__ballot(n_far != 0)) {
          const uint32_t inc = wave_incl_scan(n_far);
          uint32_t base = 0;
          if (lane() == kWave - 1) base = atomicAdd(far_count, inc);
          base = __shfl(base, kWave - 1) + inc - n_far;
#pragma unroll
          for (int r = 0; r < B; ++r)
            if (ffirst[r]) far_q[base++] = v[r];
        }
      }
    }
    __syncthreads();
  }
}

// Far-pile split (priority queue): for every pile entry and every source bit
// of its fmask, distance >= T1 stays (next pile), T0 <= distance < T1 joins
// the frontier, distance < T0 was expanded already (dropped).
__global__ __launch_bounds__(256) void k_msssp_refill(
    const int32_t* __restrict__ pile, const uint32_t* __restrict__ n_pile,
    int32_t* __restrict__ pile_next, uint32_t* __restrict__ n_pile_next,
    const u64* __restrict__ keys, int KS, uint32_t* __restrict__ fmask,
    uint32_t* __restrict__ amask, uint32_t T0, uint32_t T1, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  const int64_t n = *n_pile;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < n; b0 += stride) {
    const int64_t i = b0 + threadIdx.x;
    int32_t v = 0;
    uint32_t act = 0, keep = 0;
    if (i < n) {
      v = pile[i];
      const uint32_t m = fmask[v];
      for (uint32_t b = m; b; b &= b - 1) {
        const int sI = __ffs(b) - 1;
        const uint32_t d = (uint32_t)(keys[(int64_t)v * KS + sI] >> 32);
        if (d >= T1) keep |= 1u << sI;
        else if (d >= T0) act |= 1u << sI;
      }
      fmask[v] = keep;
      if (act) amask[v] = act;
    }
    const uint32_t a = block_append<256>(act ? 1u : 0u, out_count);
    if (act) out_q[a] = v;
    const uint32_t k = block_append<256>(keep ? 1u : 0u, n_pile_next);
    if (keep) pile_next[k] = v;
  }
}

// keys = no path (~0), masks = 0, then the sources: key (0, -1) and the
// source's bit in amask; the distinct source vertices form frontier 0.
__global__ __launch_bounds__(256) void k_msssp_init(u64* __restrict__ keys, int KS,
                                                    uint32_t* __restrict__ amask,
                                                    uint32_t* __restrict__ nmask,
                                                    uint32_t* __restrict__ fmask,
                                                    uint32_t* __restrict__ relaxed, int64_t V) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n = V * KS;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    keys[i] = ~0ull;
    if (relaxed) relaxed[i] = 0u;
    if (i < V) {
      amask[i] = 0u;
      nmask[i] = 0u;
      fmask[i] = 0u;
    }
  }
}

__global__ __launch_bounds__(64) void k_msssp_seed(const int32_t* __restrict__ src, int32_t k,
                                                   int KS, u64* __restrict__ keys,
                                                   uint32_t* __restrict__ amask) {
  const int s = threadIdx.x;
  if (s < k) {
    const int32_t v = src[s];
    keys[(int64_t)v * KS + s] = 0xffffffffull;  // distance 0, predecessor -1
    atomicOr(&amask[v], 1u << s);
  }
}

__global__ __launch_bounds__(256) void k_msssp_clear(const int32_t* __restrict__ q,
                                                     const uint32_t* __restrict__ n,
                                                     uint32_t* __restrict__ amask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)*n) amask[q[i]] = 0u;
}

// Every workgroup thread calls block_append once, so no early return.
__global__ __launch_bounds__(256) void k_msssp_move(const int32_t* __restrict__ q,
                                                    const uint32_t* __restrict__ n,
                                                    uint32_t* __restrict__ amask,
                                                    uint32_t* __restrict__ nmask,
                                                    const u64* __restrict__ keys, int KS,
                                                    uint32_t* __restrict__ relaxed,
                                                    int32_t* __restrict__ out_q,
                                                    uint32_t* __restrict__ out_count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t v = 0;
  uint32_t nm = 0;
  if (i < (int64_t)*n) {
    v = q[i];
    nm = nmask[v];
    nmask[v] = 0u;
    if (relaxed) {
      for (uint32_t b = nm; b; b &= b - 1) {
        const int sI = __ffs(b) - 1;
        const int64_t x = (int64_t)v * KS + sI;
        const uint32_t r = relaxed[x];
        if (r == (uint32_t)(keys[x] >> 32) + 1u) nm &= ~(1u << sI);
        else if (r) relaxed[x] = 0u;
      }
    }
    amask[v] = nm;
  }
  const uint32_t a = block_append<256>(nm ? 1u : 0u, out_count);
  if (nm) out_q[a] = v;
}

// dist[s][v] / pred[s][v] at caller ids for the k sources of the pass, and the
// sum over sources of the degrees of their reached vertices.
__global__ __launch_bounds__(256) void k_msssp_finalize(const u64* __restrict__ keys, int KS,
                                                        int32_t k, const int32_t* __restrict__ R,
                                                        int64_t V, uint32_t* __restrict__ dist,
                                                        int32_t* __restrict__ pred,
                                                        const int32_t* __restrict__ perm,
                                                        int64_t* __restrict__ reached_edges) {
  __shared__ int64_t s[256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t acc = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += stride) {
    const int64_t o = perm ? perm[v] : v;
    const int64_t deg = (int64_t)R[v + 1] - R[v];
    for (int sI = 0; sI < k; ++sI) {
      const u64 key = keys[v * KS + sI];
      const uint32_t d = (uint32_t)(key >> 32);
      dist[(int64_t)sI * V + o] = d;
      if (pred) pred[(int64_t)sI * V + o] = (int32_t)(uint32_t)(key & 0xffffffffull);
      if (d != 0xffffffffu) acc += deg;
    }
  }
  acc = wave_sum(acc);
  if (lane() == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < 256 / kWave; ++i) t += s[i];
    if (t) atomicAdd((unsigned long long*)reached_edges, (unsigned long long)t);
  }
}

// A source has no predecessor; a zero-weight edge into it may have tied its
// distance 0 with a smaller (distance, predecessor) key.
__global__ __launch_bounds__(64) void k_msssp_source_pred(const int32_t* __restrict__ src_orig,
                                                          int32_t k, int64_t V,
                                                          int32_t* __restrict__ pred) {
  const int s = threadIdx.x;
  if (s < k) pred[(int64_t)s * V + src_orig[s]] = -1;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <bool PQ>
hipError_t relax_n(int chunk, unsigned g, const int32_t* frontier, const int32_t* offsets,
                   const int32_t* rstart, const int32_t* chunk_start, int32_t n_f, int32_t m_f,
                   const int32_t* C, const uint32_t* W, int KS, u64* keys, const uint32_t* amask,
                   uint32_t* nmask, uint32_t* fmask, int32_t* far_q, uint32_t* far_count,
                   uint32_t T, const int32_t* perm, uint32_t* relaxed, int32_t* out_q,
                   uint32_t* out_count, hipStream_t st) {
#define GR_MS_RELAX(CH)                                                                        \
  k_msssp_relax<CH, PQ><<<g, 256, 0, st>>>(frontier, offsets, rstart, chunk_start, n_f, m_f, C, \
                                           W, KS, keys, amask, nmask, fmask, far_q, far_count,   \
                                           T, perm, relaxed, out_q, out_count)
  if (chunk == 512) GR_MS_RELAX(512);
  else if (chunk == 2048) GR_MS_RELAX(2048);
  else GR_MS_RELAX(1024);
#undef GR_MS_RELAX
  return hipGetLastError();
}

}  // namespace

int msssp_row(int k) { return k <= 4 ? 4 : (k <= 8 ? 8 : 16); }

int msssp_chunk(int chunk) { return chunk == 512 || chunk == 2048 ? chunk : 1024; }

hipError_t launch_msssp_init(u64* keys, int KS, uint32_t* amask, uint32_t* nmask, uint32_t* fmask,
                             uint32_t* relaxed, int64_t V, const int32_t* src_dev, int32_t k,
                             hipStream_t st) {
  int64_t g = blocks_for(V * KS, 256);
  if (g > 8192) g = 8192;
  k_msssp_init<<<(unsigned)g, 256, 0, st>>>(keys, KS, amask, nmask, fmask, relaxed, V);
  k_msssp_seed<<<1, 64, 0, st>>>(src_dev, k, KS, keys, amask);
  return hipGetLastError();
}

hipError_t launch_msssp_relax(int KS, int chunk, const int32_t* frontier, const int32_t* offsets,
                              const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                              int64_t m_f, const int32_t* C, const uint32_t* W, u64* keys,
                              const uint32_t* amask, uint32_t* nmask, const MsFar* far,
                              const int32_t* perm, uint32_t* relaxed, int32_t* out_q,
                              uint32_t* out_count, hipStream_t st) {
  if (n_f <= 0 || m_f <= 0) return hipSuccess;
  const int ch = msssp_chunk(chunk);
  const unsigned g = blocks_for(m_f, ch);
  if (far)
    return relax_n<true>(ch, g, frontier, offsets, rstart, chunk_start, (int32_t)n_f, (int32_t)m_f,
                         C, W, KS, keys, amask, nmask, far->fmask, far->pile, far->pile_count,
                         far->T, perm, relaxed, out_q, out_count, st);
  return relax_n<false>(ch, g, frontier, offsets, rstart, chunk_start, (int32_t)n_f, (int32_t)m_f,
                        C, W, KS, keys, amask, nmask, nullptr, nullptr, nullptr, 0u, perm, relaxed,
                        out_q, out_count, st);
}

hipError_t launch_msssp_refill(const int32_t* pile, const uint32_t* n_pile, int64_t max_pile,
                               int32_t* pile_next, uint32_t* n_pile_next, const u64* keys, int KS,
                               uint32_t* fmask, uint32_t* amask, uint32_t T0, uint32_t T1,
                               int32_t* out_q, uint32_t* out_count, hipStream_t st) {
  if (max_pile <= 0) return hipSuccess;
  int64_t g = blocks_for(max_pile, 256);
  if (g > 2048) g = 2048;
  k_msssp_refill<<<(unsigned)g, 256, 0, st>>>(pile, n_pile, pile_next, n_pile_next, keys, KS,
                                              fmask, amask, T0, T1, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_msssp_rotate(const int32_t* cur_q, const uint32_t* cur_n, int64_t max_cur,
                               const int32_t* next_q, const uint32_t* next_n, int64_t max_next,
                               uint32_t* amask, uint32_t* nmask, const u64* keys, int KS,
                               uint32_t* relaxed, int32_t* out_q, uint32_t* out_count,
                               hipStream_t st) {
  if (max_cur > 0) k_msssp_clear<<<blocks_for(max_cur, 256), 256, 0, st>>>(cur_q, cur_n, amask);
  if (max_next > 0)
    k_msssp_move<<<blocks_for(max_next, 256), 256, 0, st>>>(next_q, next_n, amask, nmask, keys, KS,
                                                            relaxed, out_q, out_count);
  return hipGetLastError();
}

hipError_t launch_msssp_finalize(const u64* keys, int KS, int32_t k, const int32_t* R, int64_t V,
                                 uint32_t* dist, int32_t* pred, const int32_t* perm,
                                 const int32_t* src_orig_dev, int64_t* reached_edges,
                                 hipStream_t st) {
  unsigned g = blocks_for(V, 256);
  if (g > 1024) g = 1024;
  k_msssp_finalize<<<g, 256, 0, st>>>(keys, KS, k, R, V, dist, pred, perm, reached_edges);
  if (pred) k_msssp_source_pred<<<1, 64, 0, st>>>(src_orig_dev, k, V, pred);
  return hipGetLastError();
}

}  // namespace gr
