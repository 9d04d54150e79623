// Device-side building blocks for gfx950 (CDNA4, 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gr {

constexpr int kWave = 64;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Number of set bits of `m` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wave-aggregated append: every active lane with `pred` gets a distinct slot
// in a global queue whose tail is `*counter`; one atomic per wavefront.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred) {
  uint64_t m = __ballot(pred);
  uint32_t base = 0;
  if (m != 0) {
    int leader = __ffsll((unsigned long long)m) - 1;
    if (lane() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
  }
  return base + lanes_below(m);
}

// Inclusive prefix sum across the wavefront (all 64 lanes must be active).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x);

// Workgroup-aggregated append: every thread contributes n slots; one atomic
// per workgroup reserves them all in the queue whose tail is *counter.
// Returns the thread's first slot.  Every thread of the workgroup must call
// it (it synchronises the workgroup).
template <int BLOCK>
__device__ __forceinline__ uint32_t block_append(uint32_t n, uint32_t* counter) {
  constexpr int NW = BLOCK / kWave;
  __shared__ uint32_t s_w[NW + 1];
  const uint32_t inc = wave_incl_scan(n);
  const int w = threadIdx.x / kWave;
  if (lane() == kWave - 1) s_w[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int i = 0; i < NW; ++i) {
      const uint32_t c = s_w[i];
      s_w[i] = t;
      t += c;
    }
    s_w[NW] = t ? atomicAdd(counter, t) : 0u;
  }
  __syncthreads();
  const uint32_t base = s_w[NW] + s_w[w] + inc - n;
  __syncthreads();  // s_w is reused by the next call
  return base;
}

// The marks of vertices 32 w .. 32 w + 31 as a bit mask; the marks are
// cleared (they are all zero again when the pass is done).
__device__ __forceinline__ uint32_t take_marks(uint8_t* __restrict__ marks, int64_t w, int64_t V) {
  const int64_t n_words = (V + 31) / 32;
  uint32_t mask = 0;
  if (w >= n_words) return 0;
  const int64_t v0 = w * 32;
  if (v0 + 32 <= V) {
    const uint4* m4 = reinterpret_cast<const uint4*>(marks + v0);
    const uint4 a = m4[0], b = m4[1];
    const uint32_t q[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((q[i] >> (8 * k)) & 0xffu) mask |= 1u << (4 * i + k);
    if (mask) {
      uint4* z = reinterpret_cast<uint4*>(marks + v0);
      z[0] = make_uint4(0, 0, 0, 0);
      z[1] = make_uint4(0, 0, 0, 0);
    }
  } else {
    for (int64_t v = v0; v < V; ++v)
      if (marks[v]) {
        mask |= 1u << (v - v0);
        marks[v] = 0;
      }
  }
  return mask;
}

// Appends the vertices 32 w + b, for every bit b of mask, to out_q with one
// atomic per workgroup (ascending within the workgroup).
// Every thread of the workgroup must call it.
template <int BLOCK>
__device__ __forceinline__ void append_mask(uint32_t mask, int64_t w, int32_t* __restrict__ out_q,
                                            uint32_t* out_count) {
  uint32_t base = block_append<BLOCK>(__popc(mask), out_count);
  while (mask) {
    const int b = __ffs(mask) - 1;
    mask &= mask - 1;
    out_q[base++] = (int32_t)(w * 32 + b);
  }
}

// Inclusive prefix sum across the wavefront (all 64 lanes must be active).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o);
    if (lane() >= o) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o);
    x = y > x ? y : x;
  }
  return x;
}

// Exclusive prefix sum over a workgroup of BLOCK threads (all active).
// `wave_tot` must hold BLOCK/64 + 1 entries of shared memory.  Returns the
// exclusive prefix of the calling thread; *total receives the block total.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* wave_tot, T* total) {
  constexpr int NW = BLOCK / kWave;
  const int w = threadIdx.x / kWave;
  T inc = wave_incl_scan(x);
  if (lane() == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < NW; ++i) {
      T t = wave_tot[i];
      wave_tot[i] = run;
      run += t;
    }
    wave_tot[NW] = run;
  }
  __syncthreads();
  T r = wave_tot[w] + inc - x;
  *total = wave_tot[NW];
  __syncthreads();
  return r;
}

// Largest index i in [lo, hi] with a[i] <= key (a ascending, a[lo] <= key).
template <typename T, typename K>
__device__ __forceinline__ int upper_index(const T* a, int lo, int hi, K key) {
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((K)a[mid] <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool bm_test(const uint32_t* bm, int32_t v) {
  return (bm[v >> 5] >> (v & 31)) & 1u;
}

}  // namespace gr
