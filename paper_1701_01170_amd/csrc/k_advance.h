// Push-advance kernels, templated on a visit functor that is fused into the
// expansion (Sec. 5.3: functors compiled into the operator kernels, and the
// filter fused with the advance so that no intermediate edge frontier is
// written).  A functor provides
//   int32_t seg_payload(int32_t u)            per-source value (e.g. dist[u])
//   void    on_frontier(int32_t u)            once per frontier vertex
//   bool    visit(u, payload, v, e)           true => append v to the output
// Three workload mappings (Sec. 5.1):
//   k_push_lb    - output-frontier load balance: equal edge chunks per
//                  workgroup over the degree prefix sum, source found by a
//                  binary search of the chunk's offsets staged in LDS;
//   k_push_light - input-frontier load balance: equal frontier slices per
//                  workgroup, their degrees scanned in LDS, the slice's edges
//                  strip-mined across the workgroup;
//   k_push_twc   - dynamic grouping: lists longer than the workgroup are
//                  expanded by the whole workgroup, lists longer than a
//                  wavefront by one wavefront, the rest by a wavefront-wide
//                  scan-based gather.
#pragma once

#include "gr_internal.h"
#include "k_common.h"

namespace gr {

constexpr int kAdvBlock = 256;
constexpr int kLbCap = 2048;  // frontier segments staged in LDS per pass

template <class F>
__global__ __launch_bounds__(kAdvBlock) void k_push_lb(
    const int32_t* __restrict__ frontier, const int32_t* __restrict__ offsets, int32_t n_f,
    int32_t m_f, const int32_t* __restrict__ R, const int32_t* __restrict__ C, F f,
    int32_t* __restrict__ out_q, uint32_t* __restrict__ out_count, int32_t chunk) {
  __shared__ int32_t s_off[kLbCap + 1];
  __shared__ int32_t s_u[kLbCap];
  __shared__ int32_t s_rb[kLbCap];
  __shared__ int32_t s_pay[kLbCap];
  __shared__ int32_t s_rng[2];
  const int64_t e0 = (int64_t)blockIdx.x * chunk;
  if (e0 >= m_f) return;
  const int64_t e1 = e0 + chunk < m_f ? e0 + chunk : m_f;
  if (threadIdx.x == 0) {
    s_rng[0] = upper_index(offsets, 0, n_f - 1, e0);
    s_rng[1] = upper_index(offsets, 0, n_f - 1, e1 - 1);
  }
  __syncthreads();
  const int sb = s_rng[0], se = s_rng[1];
  for (int pb = sb; pb <= se; pb += kLbCap) {
    const int cnt = (se - pb + 1) < kLbCap ? (se - pb + 1) : kLbCap;
    for (int i = threadIdx.x; i < cnt; i += kAdvBlock) {
      const int s = pb + i;
      const int32_t u = frontier[s];
      s_off[i] = offsets[s];
      s_u[i] = u;
      s_rb[i] = R[u];
      s_pay[i] = f.seg_payload(u);
    }
    if (threadIdx.x == 0) s_off[cnt] = offsets[pb + cnt];
    __syncthreads();
    const int64_t lo = e0 > (int64_t)s_off[0] ? e0 : (int64_t)s_off[0];
    const int64_t hi = e1 < (int64_t)s_off[cnt] ? e1 : (int64_t)s_off[cnt];
    for (int64_t e = lo + threadIdx.x; e < hi; e += kAdvBlock) {
      const int k = upper_index(s_off, 0, cnt - 1, e);
      const int32_t u = s_u[k];
      const int64_t ce = (int64_t)s_rb[k] + (e - s_off[k]);
      const int32_t v = C[ce];
      const bool app = f.visit(u, s_pay[k], v, ce);
      const uint32_t slot = wave_append(out_count, app);
      if (app) out_q[slot] = v;
    }
    __syncthreads();
  }
}

template <class F>
__global__ __launch_bounds__(kAdvBlock) void k_push_light(
    const int32_t* __restrict__ frontier, int32_t n_f, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, F f, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  __shared__ int32_t s_off[kAdvBlock];
  __shared__ int32_t s_u[kAdvBlock];
  __shared__ int32_t s_rb[kAdvBlock];
  __shared__ int32_t s_pay[kAdvBlock];
  __shared__ int64_t s_tot[kAdvBlock / kWave + 1];
  const int64_t i = (int64_t)blockIdx.x * kAdvBlock + threadIdx.x;
  int32_t u = 0, rb = 0, d = 0, pay = 0;
  if (i < n_f) {
    u = frontier[i];
    rb = R[u];
    d = R[u + 1] - rb;
    pay = f.seg_payload(u);
    f.on_frontier(u);
  }
  int64_t total;
  const int64_t ex = block_excl_scan<kAdvBlock>((int64_t)d, s_tot, &total);
  s_off[threadIdx.x] = (int32_t)ex;
  s_u[threadIdx.x] = u;
  s_rb[threadIdx.x] = rb;
  s_pay[threadIdx.x] = pay;
  __syncthreads();
  for (int64_t e = threadIdx.x; e < total; e += kAdvBlock) {
    const int k = upper_index(s_off, 0, kAdvBlock - 1, e);
    const int64_t ce = (int64_t)s_rb[k] + (e - s_off[k]);
    const int32_t v = C[ce];
    const bool app = f.visit(s_u[k], s_pay[k], v, ce);
    const uint32_t slot = wave_append(out_count, app);
    if (app) out_q[slot] = v;
  }
}

template <class F>
__global__ __launch_bounds__(kAdvBlock) void k_push_twc(
    const int32_t* __restrict__ frontier, int32_t n_f, const int32_t* __restrict__ R,
    const int32_t* __restrict__ C, F f, int32_t* __restrict__ out_q,
    uint32_t* __restrict__ out_count) {
  constexpr int NW = kAdvBlock / kWave;
  __shared__ int32_t s_claim;
  __shared__ int32_t s_cu, s_crb, s_cd, s_cpay;
  __shared__ int32_t s_woff[NW][kWave];
  __shared__ int32_t s_wu[NW][kWave];
  __shared__ int32_t s_wrb[NW][kWave];
  __shared__ int32_t s_wpay[NW][kWave];
  const int64_t i = (int64_t)blockIdx.x * kAdvBlock + threadIdx.x;
  const int w = threadIdx.x / kWave;
  int32_t u = 0, rb = 0, d = 0, pay = 0;
  if (i < n_f) {
    u = frontier[i];
    rb = R[u];
    d = R[u + 1] - rb;
    pay = f.seg_payload(u);
    f.on_frontier(u);
  }
  // workgroup tier: lists longer than the workgroup
  bool big = d > kAdvBlock;
  for (;;) {
    if (threadIdx.x == 0) s_claim = -1;
    __syncthreads();
    if (big) s_claim = threadIdx.x;
    __syncthreads();
    const int c = s_claim;
    if (c < 0) break;
    if (c == (int)threadIdx.x) {
      s_cu = u;
      s_crb = rb;
      s_cd = d;
      s_cpay = pay;
      big = false;
    }
    __syncthreads();
    const int32_t cu = s_cu, crb = s_crb, cd = s_cd, cpay = s_cpay;
    for (int j = threadIdx.x; j < cd; j += kAdvBlock) {
      const int64_t ce = (int64_t)crb + j;
      const int32_t v = C[ce];
      const bool app = f.visit(cu, cpay, v, ce);
      const uint32_t slot = wave_append(out_count, app);
      if (app) out_q[slot] = v;
    }
    __syncthreads();
  }
  // wavefront tier: lists longer than a wavefront
  uint64_t med = __ballot(d > kWave && d <= kAdvBlock);
  while (med) {
    const int l = __ffsll((unsigned long long)med) - 1;
    med &= med - 1;
    const int32_t cu = __shfl(u, l), crb = __shfl(rb, l), cd = __shfl(d, l), cpay = __shfl(pay, l);
    for (int j = lane(); j < cd; j += kWave) {
      const int64_t ce = (int64_t)crb + j;
      const int32_t v = C[ce];
      const bool app = f.visit(cu, cpay, v, ce);
      const uint32_t slot = wave_append(out_count, app);
      if (app) out_q[slot] = v;
    }
  }
  // lane tier: scan-based gather of the short lists across the wavefront
  const int32_t ds = d <= kWave ? d : 0;
  const int32_t inc = wave_incl_scan(ds);
  const int32_t tot = __shfl(inc, kWave - 1);
  s_woff[w][lane()] = inc - ds;
  s_wu[w][lane()] = u;
  s_wrb[w][lane()] = rb;
  s_wpay[w][lane()] = pay;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (int e = lane(); e < tot; e += kWave) {
    const int k = upper_index(s_woff[w], 0, kWave - 1, e);
    const int64_t ce = (int64_t)s_wrb[w][k] + (e - s_woff[w][k]);
    const int32_t v = C[ce];
    const bool app = f.visit(s_wu[w][k], s_wpay[w][k], v, ce);
    const uint32_t slot = wave_append(out_count, app);
    if (app) out_q[slot] = v;
  }
}

}  // namespace gr
