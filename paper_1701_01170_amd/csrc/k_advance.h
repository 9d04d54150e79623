// Push-advance kernels, templated on a visit functor that is fused into the
// expansion (Sec. 5.3: functors compiled into the operator kernels, and the
// filter fused with the advance so that no intermediate edge frontier is
// written).  A functor provides
//   pay_t    seg_payload(int32_t u)          per-source value (e.g. dist[u]);
//                                            pay_t is the functor's payload type
//   uint32_t edge_value(int64_t e)           per-edge value (e.g. weight)
//   bool     probe(u, payload, v, ev)        read-only test: may the edge update v?
//   bool     commit(u, payload, v, ev)       atomic update; true => append v
//   kFar                                     true for functors whose commit
//                                            returns 0 / 1 / 2: 2 appends v to
//                                            a second queue (f.far_q, f.far_count)
//   seg_note(u, payload)                     optional: told each frontier vertex's
//                                            payload as its edges are staged
//   kBatchCommit                             true for functors that provide
//                                            commit_batch<B>(u, pay, v, ev, ok, code):
//                                            the commits of a lane's B edges in
//                                            phases, so that their atomics are in
//                                            flight together instead of one
//                                            round trip after another
// Edges are handled in batches: every lane first issues all of its
// column-index loads, then all probe loads, then the atomics of the edges
// that survive, then one wavefront-aggregated append; independent loads are
// in flight together instead of one dependent chain per edge.
//
// Three workload mappings (Sec. 5.1):
//   k_push_lb    - output-frontier load balance: equal edge chunks per
//                  workgroup; the chunk -> first-segment map is scattered by
//                  the offsets kernel (the sorted search of 0, N, 2N, ... in the
//                  degree prefix sum), and each edge finds its segment with an
//                  LDS max-scan of segment starts;
//   k_push_light - input-frontier load balance: equal frontier slices per
//                  workgroup, degrees scanned in LDS, the slice's edges
//                  strip-mined across the workgroup;
//   k_push_twc   - dynamic grouping: lists longer than the workgroup are
//                  expanded by the whole workgroup, lists longer than a
//                  wavefront by one wavefront, the rest by a wavefront-wide
//                  scan-based gather.
#pragma once

#include <type_traits>
#include <utility>

#include "gr_internal.h"
#include "k_common.h"

namespace gr {

// Optional functor members.  block_init(): per-workgroup state (e.g. an LDS
// table), run once by every thread before the first edge, followed by a
// workgroup barrier.  out_cap: the output queue holds this many entries;
// appends beyond it are counted in *out_count but not stored.
template <class F, class = void>
struct has_block_init : std::false_type {};
template <class F>
struct has_block_init<F, std::void_t<decltype(std::declval<const F&>().block_init())>>
    : std::true_type {};
template <class F, class = void>
struct has_out_cap : std::false_type {};
template <class F>
struct has_out_cap<F, std::void_t<decltype(&F::out_cap)>> : std::true_type {};

template <class F, class = void>
struct has_seg_note : std::false_type {};
template <class F>
struct has_seg_note<F, std::void_t<decltype(std::declval<const F&>().seg_note(
                           0, std::declval<typename F::pay_t>()))>> : std::true_type {};

// seg_note(u, payload): told the payload a frontier vertex's edges are about
// to be processed with (once per vertex and chunk of its row).
template <class F>
__device__ __forceinline__ void functor_seg_note(const F& f, int32_t u,
                                                 const typename F::pay_t& pay) {
  if constexpr (has_seg_note<F>::value) f.seg_note(u, pay);
}

template <class F>
__device__ __forceinline__ void functor_block_init(const F& f) {
  if constexpr (has_block_init<F>::value) {
    f.block_init();
    __syncthreads();
  }
}

// out_q[slot] = v, unless the functor bounds its queue and slot is past it.
template <class F>
__device__ __forceinline__ void put_out(const F& f, int32_t* __restrict__ out_q, uint32_t slot,
                                        int32_t v) {
  if constexpr (has_out_cap<F>::value) {
    if (slot < f.out_cap) out_q[slot] = v;
  } else {
    out_q[slot] = v;
  }
}

constexpr int kAdvBlock = 256;
// Frontier segments a workgroup stages in LDS per pass: half the chunk's
// edges (at most 2048).  A chunk whose rows average fewer than two edges takes
// more than one pass; a smaller stage leaves LDS for more resident workgroups.
constexpr int lb_cap(int chunk_edges) {
  return chunk_edges / 2 < 256 ? 256 : (chunk_edges / 2 > 2048 ? 2048 : chunk_edges / 2);
}

// Process up to B edges per lane: ok[r] marks a real edge (u[r], pay[r], ce[r]).
// All 64 lanes must take part.  With AGG the whole workgroup appends with one
// atomic (every thread of the workgroup must then call it the same number of
// times): a single queue tail shared by the whole grid serialises its
// atomics, so fewer of them is the point.
template <class F, int B, bool AGG = false, int BLOCK = kAdvBlock>
__device__ __forceinline__ void edge_batch(const F& f, const int32_t* __restrict__ C, bool (&ok)[B],
                                           const int32_t (&u)[B], const typename F::pay_t (&pay)[B],
                                           const int32_t (&ce)[B], int32_t* __restrict__ out_q,
                                           uint32_t* __restrict__ out_count) {
  int32_t v[B];
  uint32_t ev[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    v[r] = ok[r] ? C[ce[r]] : 0;
    ev[r] = ok[r] ? f.edge_value(ce[r]) : 0u;
  }
#pragma unroll
  for (int r = 0; r < B; ++r) ok[r] = ok[r] && f.probe(u[r], pay[r], v[r], ev[r]);
  uint32_t n_app = 0, n_far = 0;
  bool far[B];
  int code[B];
  if constexpr (F::kBatchCommit) {
    f.template commit_batch<B>(u, pay, v, ev, ok, code);
  } else {
#pragma unroll
    for (int r = 0; r < B; ++r) code[r] = ok[r] ? (int)f.commit(u[r], pay[r], v[r], ev[r]) : 0;
  }
#pragma unroll
  for (int r = 0; r < B; ++r) {
    const int c = code[r];
    ok[r] = c == 1;
    far[r] = F::kFar && c == 2;
    n_app += ok[r] ? 1u : 0u;
    n_far += far[r] ? 1u : 0u;
  }
  if constexpr (F::kFar) {
    if (__ballot(n_far != 0)) {
      const uint32_t finc = wave_incl_scan(n_far);
      uint32_t fbase = 0;
      if (lane() == kWave - 1) fbase = atomicAdd(f.far_count, finc);
      fbase = __shfl(fbase, kWave - 1) + finc - n_far;
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (far[r]) f.far_q[fbase++] = v[r];
    }
  }
  if constexpr (AGG) {
    uint32_t base = block_append<BLOCK>(n_app, out_count);
#pragma unroll
    for (int r = 0; r < B; ++r)
      if (ok[r]) put_out(f, out_q, base++, v[r]);
  } else {
    // wavefront-aggregated append of every lane's survivors
    const uint64_t any = __ballot(n_app != 0);
    if (any == 0) return;
    const uint32_t inc = wave_incl_scan(n_app);
    uint32_t base = 0;
    if (lane() == kWave - 1) base = atomicAdd(out_count, inc);
    base = __shfl(base, kWave - 1) + inc - n_app;
#pragma unroll
    for (int r = 0; r < B; ++r)
      if (ok[r]) put_out(f, out_q, base++, v[r]);
  }
}

// Inclusive max-scan over s_seg[0, SPT * BLOCK) in place, SPT consecutive
// slots per thread: turns the scattered segment starts into each edge slot's
// segment index.  s_tmp holds BLOCK / kWave + 1 entries.  Every thread of the
// workgroup calls it (one barrier inside); the caller adds the barrier after.
template <int SPT, int BLOCK>
__device__ __forceinline__ void lb_seg_maxscan(uint16_t* s_seg, int32_t* s_tmp) {
  int32_t run = 0;
  for (int r = 0; r < SPT; ++r) {
    const int32_t x = s_seg[threadIdx.x * SPT + r];
    run = x > run ? x : run;
  }
  int32_t inc = run;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(inc, o);
    if (lane() >= o) inc = y > inc ? y : inc;
  }
  if (lane() == kWave - 1) s_tmp[threadIdx.x / kWave] = inc;
  __syncthreads();
  int32_t ex = 0;
  for (int i = 0; i < (int)threadIdx.x / kWave; ++i) ex = s_tmp[i] > ex ? s_tmp[i] : ex;
  int32_t wx = __shfl_up(inc, 1);
  if (lane() == 0) wx = 0;
  run = wx > ex ? wx : ex;
  for (int r = 0; r < SPT; ++r) {
    const int32_t x = s_seg[threadIdx.x * SPT + r];
    run = x > run ? x : run;
    s_seg[threadIdx.x * SPT + r] = (uint16_t)run;
  }
}

// One workgroup per chunk of NB * EPT * 256 edges of the output frontier
// (its edges are positions e_base .. e_base + m_f - 1 of `offsets`, normally
// from 0; a frontier inside a longer scanned list starts further on).  The
// frontier segments overlapping the chunk are staged in LDS (lb_cap per pass);
// a 16-bit segment index per edge slot comes from scattering segment starts and
// a max-scan; the edges are then processed in NB batches of EPT per thread
// (EPT independent loads in flight per lane).
template <class F, int EPT, int NB, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_push_lb(
    const int32_t* __restrict__ frontier, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ rstart, const int32_t* __restrict__ chunk_start, int32_t n_f,
    int32_t m_f, const int32_t* __restrict__ C, F f,
    int32_t* __restrict__ out_q, uint32_t* __restrict__ out_count, int64_t e_base) {
  constexpr int BATCH = BLOCK * EPT;
  constexpr int N = BATCH * NB;
  constexpr int SPT = N / BLOCK;  // segment-map slots per thread
  constexpr int CAP = lb_cap(N);
  __shared__ uint16_t s_seg[N];
  __shared__ int32_t s_off[CAP + 1];
  __shared__ int32_t s_u[CAP];
  __shared__ int32_t s_rb[CAP];
  __shared__ typename F::pay_t s_pay[CAP];
  __shared__ int32_t s_tmp[BLOCK / kWave + 1];
  functor_block_init(f);
  const int c = blockIdx.x;
  const int64_t e0 = e_base + (int64_t)c * N;
  const int64_t e1 = e0 + N < e_base + m_f ? e0 + N : e_base + m_f;
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
      const typename F::pay_t pu = f.seg_payload(u);
      s_pay[i] = pu;
      functor_seg_note(f, u, pu);
    }
    if (threadIdx.x == 0) s_off[cnt] = offsets[pb + cnt];
    for (int j = threadIdx.x; j < N; j += BLOCK) s_seg[j] = 0;
    __syncthreads();
    const int64_t lo = e0 > (int64_t)s_off[0] ? e0 : (int64_t)s_off[0];
    const int64_t hi = e1 < (int64_t)s_off[cnt] ? e1 : (int64_t)s_off[cnt];
    // starts of the non-empty segments inside [lo, hi) (exactly one non-empty
    // segment starts at any edge position; empty ones own no edge)
    for (int k = 1 + threadIdx.x; k < cnt; k += BLOCK) {
      const int64_t pos = (int64_t)s_off[k] - lo;
      if (pos < hi - lo && s_off[k + 1] > s_off[k]) s_seg[pos] = (uint16_t)k;
    }
    __syncthreads();
    lb_seg_maxscan<SPT, BLOCK>(s_seg, s_tmp);
    __syncthreads();
    for (int b = 0; b < NB; ++b) {
      if (lo + (int64_t)b * BATCH >= hi) break;
      bool ok[EPT];
      int32_t u[EPT];
      typename F::pay_t pay[EPT];
      int32_t ce[EPT];
#pragma unroll
      for (int r = 0; r < EPT; ++r) {
        const int j = b * BATCH + r * BLOCK + threadIdx.x;
        const int64_t e = lo + j;
        ok[r] = e < hi;
        const int k = ok[r] ? (int)s_seg[j] : 0;
        u[r] = s_u[k];
        pay[r] = s_pay[k];
        ce[r] = s_rb[k] + (int32_t)(e - s_off[k]);
      }
      edge_batch<F, EPT, true, BLOCK>(f, C, ok, u, pay, ce, out_q, out_count);
    }
    __syncthreads();
  }
}

template <class F, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_push_light(
    const int32_t* __restrict__ frontier, int32_t n_f, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, F f, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  constexpr int B = 4;
  __shared__ int32_t s_off[BLOCK];
  __shared__ int32_t s_u[BLOCK];
  __shared__ int32_t s_rb[BLOCK];
  __shared__ typename F::pay_t s_pay[BLOCK];
  __shared__ int64_t s_tot[BLOCK / kWave + 1];
  functor_block_init(f);
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  int32_t u0 = 0, rb = 0, d = 0;
  typename F::pay_t pay0 = 0;
  if (i < n_f) {
    u0 = frontier[i];
    rb = R[u0];
    d = R[u0 + 1] - rb;
    pay0 = f.seg_payload(u0);
    functor_seg_note(f, u0, pay0);
  }
  int64_t total;
  const int64_t ex = block_excl_scan<BLOCK>((int64_t)d, s_tot, &total);
  s_off[threadIdx.x] = (int32_t)ex;
  s_u[threadIdx.x] = u0;
  s_rb[threadIdx.x] = rb;
  s_pay[threadIdx.x] = pay0;
  __syncthreads();
  for (int64_t base = 0; base < total; base += (int64_t)BLOCK * B) {
    bool ok[B];
    int32_t u[B];
    typename F::pay_t pay[B];
    int32_t ce[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int64_t e = base + r * BLOCK + threadIdx.x;
      ok[r] = e < total;
      const int k = ok[r] ? upper_index(s_off, 0, BLOCK - 1, e) : 0;
      u[r] = s_u[k];
      pay[r] = s_pay[k];
      ce[r] = s_rb[k] + (int32_t)(e - s_off[k]);
    }
    edge_batch<F, B, true, BLOCK>(f, C, ok, u, pay, ce, out_q, out_count);
  }
}

// TWC tiers: lists longer than block_min are expanded by the whole
// workgroup, lists longer than wave_min by one wavefront, the rest by the
// lane-tier gather (0 <= wave_min <= block_min; any split is correct).
template <class F, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_push_twc(
    const int32_t* __restrict__ frontier, int32_t n_f, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, F f, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count, int32_t wave_min, int32_t block_min) {
  constexpr int NW = BLOCK / kWave;
  constexpr int B = 4;
  __shared__ int32_t s_claim;
  __shared__ int32_t s_cu, s_crb, s_cd;
  __shared__ typename F::pay_t s_cpay;
  __shared__ int32_t s_woff[NW][kWave];
  __shared__ int32_t s_wu[NW][kWave];
  __shared__ int32_t s_wrb[NW][kWave];
  __shared__ typename F::pay_t s_wpay[NW][kWave];
  functor_block_init(f);
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int w = threadIdx.x / kWave;
  int32_t u0 = 0, rb = 0, d = 0;
  typename F::pay_t pay0 = 0;
  if (i < n_f) {
    u0 = frontier[i];
    rb = R[u0];
    d = R[u0 + 1] - rb;
    pay0 = f.seg_payload(u0);
    functor_seg_note(f, u0, pay0);
  }
  // workgroup tier
  bool big = d > block_min;
  for (;;) {
    if (threadIdx.x == 0) s_claim = -1;
    __syncthreads();
    if (big) s_claim = threadIdx.x;
    __syncthreads();
    const int c = s_claim;
    if (c < 0) break;
    if (c == (int)threadIdx.x) {
      s_cu = u0;
      s_crb = rb;
      s_cd = d;
      s_cpay = pay0;
      big = false;
    }
    __syncthreads();
    const int32_t cu = s_cu, crb = s_crb, cd = s_cd;
    const typename F::pay_t cpay = s_cpay;
    for (int base = 0; base < cd; base += BLOCK * B) {
      bool ok[B];
      int32_t u[B];
      typename F::pay_t pay[B];
      int32_t ce[B];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const int j = base + r * BLOCK + threadIdx.x;
        ok[r] = j < cd;
        u[r] = cu;
        pay[r] = cpay;
        ce[r] = crb + j;
      }
      edge_batch<F, B>(f, C, ok, u, pay, ce, out_q, out_count);
    }
    __syncthreads();
  }
  // wavefront tier
  uint64_t med = __ballot(d > wave_min && d <= block_min);
  while (med) {
    const int l = __ffsll((unsigned long long)med) - 1;
    med &= med - 1;
    const int32_t cu = __shfl(u0, l), crb = __shfl(rb, l), cd = __shfl(d, l);
    const typename F::pay_t cpay = __shfl(pay0, l);
    for (int base = 0; base < cd; base += kWave * B) {
      bool ok[B];
      int32_t u[B];
      typename F::pay_t pay[B];
      int32_t ce[B];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const int j = base + r * kWave + lane();
        ok[r] = j < cd;
        u[r] = cu;
        pay[r] = cpay;
        ce[r] = crb + j;
      }
      edge_batch<F, B>(f, C, ok, u, pay, ce, out_q, out_count);
    }
  }
  // lane tier: scan-based gather of the short lists across the wavefront
  const int32_t ds = d <= wave_min ? d : 0;
  const int32_t inc = wave_incl_scan(ds);
  const int32_t tot = __shfl(inc, kWave - 1);
  s_woff[w][lane()] = inc - ds;
  s_wu[w][lane()] = u0;
  s_wrb[w][lane()] = rb;
  s_wpay[w][lane()] = pay0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (int base = 0; base < tot; base += kWave * B) {
    bool ok[B];
    int32_t u[B];
    typename F::pay_t pay[B];
    int32_t ce[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int e = base + r * kWave + lane();
      ok[r] = e < tot;
      const int k = ok[r] ? upper_index(s_woff[w], 0, kWave - 1, e) : 0;
      u[r] = s_wu[w][k];
      pay[r] = s_wpay[w][k];
      ce[r] = s_wrb[w][k] + (e - s_woff[w][k]);
    }
    edge_batch<F, B>(f, C, ok, u, pay, ce, out_q, out_count);
  }
}

inline unsigned adv_blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Output-balanced LB with `chunk` edges per workgroup of BLOCK threads: EPT
// edges per thread per batch (at most 32 in flight; 16 with 512 threads, whose
// waves get at most 128 vector registers), NB batches.
template <class F, int BLOCK>
inline void launch_lb(int chunk, unsigned g, const int32_t* frontier, const int32_t* offsets,
                      const int32_t* rstart, const int32_t* chunk_start, int32_t n_f, int32_t m_f,
                      const int32_t* C, const F& f, int32_t* out_q, uint32_t* out_count,
                      hipStream_t st, int64_t e_base = 0) {
#define GR_LB(CH)                                                                              \
  case CH: {                                                                                   \
    constexpr int cap = BLOCK >= 512 ? 16 : 32;                                                \
    constexpr int ept = (CH / BLOCK) < cap ? (CH / BLOCK) : cap;                               \
    constexpr int nb = CH / (BLOCK * ept);                                                     \
    k_push_lb<F, ept, nb, BLOCK><<<g, BLOCK, 0, st>>>(frontier, offsets, rstart, chunk_start,   \
                                                     n_f, m_f, C, f, out_q, out_count, e_base);  \
    break;                                                                                     \
  }
  switch (chunk) {
    GR_LB(512)
    GR_LB(1024)
    GR_LB(2048)
    GR_LB(4096)
    GR_LB(16384)
    default:
      GR_LB(8192)
  }
#undef GR_LB
}

template <class F, int BLOCK>
inline hipError_t push_dispatch_block(int mode, const int32_t* frontier, const int32_t* offsets,
                                      const int32_t* rstart, const int32_t* chunk_start,
                                      int64_t n_f, int64_t m_f, const int32_t* R,
                                      const int32_t* C, const F& f, int32_t* out_q,
                                      uint32_t* out_count, const AdvCfg& cfg, hipStream_t st,
                                      int64_t e_base) {
  if (mode == 0) {
    int32_t wmin = cfg.twc_wave_min >= 0 ? cfg.twc_wave_min : kWave;
    int32_t bmin = cfg.twc_block_min >= 0 ? cfg.twc_block_min : BLOCK;
    if (bmin < wmin) bmin = wmin;
    k_push_twc<F, BLOCK><<<adv_blocks(n_f, BLOCK), BLOCK, 0, st>>>(
        frontier, (int32_t)n_f, R, C, f, out_q, out_count, wmin, bmin);
  } else if (mode == 1) {
    k_push_light<F, BLOCK><<<adv_blocks(n_f, BLOCK), BLOCK, 0, st>>>(frontier, (int32_t)n_f, R, C,
                                                                   f, out_q, out_count);
  } else {
    if (m_f <= 0) return hipSuccess;
    launch_lb<F, BLOCK>(cfg.chunk, adv_blocks(m_f, cfg.chunk), frontier, offsets, rstart,
                        chunk_start, (int32_t)n_f, (int32_t)m_f, C, f, out_q, out_count, st,
                        e_base);
  }
  return hipGetLastError();
}

// mode: 0 = TWC, 1 = LB_LIGHT, 2 = LB with cfg.chunk edges per workgroup
// (512, 1024, 2048, 4096, 8192 or 16384; the frontier's edges at positions
// e_base .. of `offsets`); workgroups of cfg.block threads (128, 256 or 512).
template <class F>
inline hipError_t push_dispatch(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C, const F& f,
                                int32_t* out_q, uint32_t* out_count, const AdvCfg& cfg,
                                hipStream_t st, int64_t e_base = 0) {
  if (n_f <= 0) return hipSuccess;
  switch (cfg.block) {
    case 128:
      return push_dispatch_block<F, 128>(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R,
                                         C, f, out_q, out_count, cfg, st, e_base);
    case 512:
      return push_dispatch_block<F, 512>(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R,
                                         C, f, out_q, out_count, cfg, st, e_base);
    default:
      return push_dispatch_block<F, 256>(mode, frontier, offsets, rstart, chunk_start, n_f, m_f, R,
                                         C, f, out_q, out_count, cfg, st, e_base);
  }
}

}  // namespace gr
