// Device-predicated level step: one push level of BFS or SSSP for a small
// frontier, written so that many levels can be enqueued back to back with no
// host round trip in between (the per-iteration termination check of the
// bulk-synchronous loop, Sec. 4 and Sec. 5.2, moved onto the device).
//
// Every workgroup reads the same control values, all written by earlier
// kernels, and stages the same frontier, so all take the same decision: the
// level runs only if no earlier level of the block declined, the frontier is
// non-empty, it fits the LDS staging (kDlMaxN vertices) and the caller's edge
// bound, and (BFS) the direction heuristic of Sec. 5.1 would still push.  A
// declining level sets dl_stop, so the rest of the block does nothing.
//
// A running level is output-balanced like LB (Sec. 5.1): each workgroup stages
// the whole frontier in LDS, scans its degrees (which gives the level its m_f
// without a statistics pass), and expands one equal slice of the edges.
//
// Functors used here also provide prepare(ctrl, step) (the functor of this
// step, e.g. SSSP's priority-queue threshold read from the control block) and
// advance(ctrl, step, refill) (the state of the next step, written once).
// With the SSSP priority queue (kFar), a step whose frontier is empty but
// whose far pile is not becomes a refill step instead of stopping the block.
#pragma once

#include "k_advance.h"

namespace gr {

constexpr int kDlPerThread = kDlMaxN / kAdvBlock;
static_assert(kDlMaxN % kAdvBlock == 0, "frontier staging assumes whole rows");

template <class F>
__global__ __launch_bounds__(kAdvBlock) void k_dstep(DlArgs a, F f) {
  using pay_t = typename F::pay_t;
  constexpr int B = 4;
  __shared__ int32_t s_u[kDlMaxN];
  __shared__ int32_t s_rb[kDlMaxN];
  __shared__ int32_t s_off[kDlMaxN + 1];
  __shared__ pay_t s_pay[kDlMaxN];
  __shared__ int64_t s_tot[kAdvBlock / kWave + 1];
  __shared__ int64_t s_max[kAdvBlock / kWave];
  Ctrl* ctrl = a.ctrl;
  if (ctrl->dl_stop) return;
  const F fs = f.prepare(ctrl, a.step);
  const int64_t n_f = ctrl->q_count[a.cur];
  const int64_t vm = ctrl->dl_vm[a.step & 1];
  const int64_t vn = ctrl->dl_vn[a.step & 1];
  const int next = (a.cur + 1) % 3, prev = (a.cur + 2) % 3;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  bool refill = false;
  if constexpr (F::kFar) refill = n_f == 0 && fs.far_pending(ctrl);
  if (!refill && !(n_f > 0 && n_f <= a.max_n && n_f <= kDlMaxN)) {
    if (lead) ctrl->dl_stop = 1;
    return;
  }
  if constexpr (F::kFar) {
    if (refill) {
      if (lead) {
        // none of these is read by this kernel
        ctrl->dl_levels = a.step + 1;
        ctrl->q_count[prev] = 0;
        ctrl->dl_vm[(a.step + 1) & 1] = vm;
        ctrl->dl_vn[(a.step + 1) & 1] = vn;
        fs.advance(ctrl, a.step, true);
        if (a.log) {
          a.log[3 * a.step + 0] = 0;
          a.log[3 * a.step + 1] = 0;
          a.log[3 * a.step + 2] = 0;
        }
      }
      fs.refill(ctrl, a.q_next, &ctrl->q_count[next]);
      return;
    }
  }
  // every workgroup stages the whole frontier and scans its degrees
  // (kDlPerThread consecutive entries per thread); the scan total is the
  // level's frontier edge count m_f
  const int nf = (int)n_f;
  for (int j = threadIdx.x; j < nf; j += kAdvBlock) s_u[j] = a.q_cur[j];
  __syncthreads();
  const int j0 = threadIdx.x * kDlPerThread;
  int32_t d[kDlPerThread];
  int64_t sum = 0, mx = 0;
#pragma unroll
  for (int r = 0; r < kDlPerThread; ++r) {
    const int j = j0 + r;
    d[r] = 0;
    if (j < nf) {
      const int32_t u = s_u[j];
      const int32_t rb = a.R[u];
      d[r] = a.R[u + 1] - rb;
      s_rb[j] = rb;
      s_pay[j] = fs.seg_payload(u);
      sum += d[r];
      mx = d[r] > mx ? d[r] : mx;
    }
  }
  int64_t total;
  int64_t ex = block_excl_scan<kAdvBlock>(sum, s_tot, &total);
#pragma unroll
  for (int r = 0; r < kDlPerThread; ++r) {
    const int j = j0 + r;
    if (j < nf) {
      s_off[j] = (int32_t)ex;
      ex += d[r];
    }
  }
  if (threadIdx.x == 0) s_off[nf] = (int32_t)total;
  mx = wave_max(mx);
  if (lane() == 0) s_max[threadIdx.x / kWave] = mx;
  __syncthreads();
  // the level runs only within the caller's edge bound and, under the
  // heuristic, while its push test holds (Sec. 5.1 push -> pull); every
  // workgroup computes the same total, so all take the same decision
  bool run = total <= a.max_m;
  const double pull_bound = a.edges_vs_all ? (double)a.E : (double)(a.E - vm - total);
  if (run && a.do_a >= 0.0 && (double)total > pull_bound * a.do_a) run = false;
  if (!run) {
    if (lead) ctrl->dl_stop = 1;
    return;
  }
  if (lead) {
    // none of these is read by this kernel: the counter of the previous
    // frontier becomes the append target of the next level
    ctrl->dl_levels = a.step + 1;
    ctrl->q_count[prev] = 0;
    ctrl->dl_vm[(a.step + 1) & 1] = vm + total;
    ctrl->dl_vn[(a.step + 1) & 1] = vn + n_f;
    fs.advance(ctrl, a.step, false);
    if (a.log) {
      int64_t m = 0;
      for (int i = 0; i < kAdvBlock / kWave; ++i) m = s_max[i] > m ? s_max[i] : m;
      a.log[3 * a.step + 0] = n_f;
      a.log[3 * a.step + 1] = total;
      a.log[3 * a.step + 2] = m;
    }
  }
  for (int j = blockIdx.x * kAdvBlock + threadIdx.x; j < nf; j += gridDim.x * kAdvBlock)
    fs.frontier_vertex(s_u[j]);
  // equal edge slices (at least one row of the workgroup each); workgroups
  // past the last slice have nothing more to do
  const int64_t G = gridDim.x;
  int64_t per = (total + G - 1) / G;
  if (per < kAdvBlock) per = kAdvBlock;
  const int64_t lo = (int64_t)blockIdx.x * per;
  if (lo >= total) return;
  const int64_t hi = lo + per < total ? lo + per : total;
  for (int64_t base = lo; base < hi; base += (int64_t)kAdvBlock * B) {
    bool ok[B];
    int32_t u[B];
    pay_t pay[B];
    int32_t ce[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const int64_t e = base + r * kAdvBlock + threadIdx.x;
      ok[r] = e < hi;
      const int k = ok[r] ? upper_index(s_off, 0, nf - 1, (int32_t)e) : 0;
      u[r] = s_u[k];
      pay[r] = s_pay[k];
      ce[r] = s_rb[k] + (int32_t)(e - s_off[k]);
    }
    edge_batch<F, B, true>(fs, a.C, ok, u, pay, ce, a.q_next, &ctrl->q_count[next]);
  }
}

}  // namespace gr
