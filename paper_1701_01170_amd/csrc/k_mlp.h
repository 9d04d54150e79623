// Strategy-selector network shared by the inference kernels: layout of the
// flat fp32 parameter array and the workgroup-wide argmin of the predicted
// step times.  Parameters (row-major):
//   W1[32][8], b1[32], W2[32][32], b2[32], W3[4][32], b3[4]   (1476 floats).
// Outputs are predicted log2 step times of the four advance actions.
#pragma once

#include "gr_internal.h"

namespace gr {

constexpr int kIn = 8, kH = 32, kOut = 4;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kOut * kH, kNP = oB3 + kOut;
static_assert(kNP == GR_MLP_N_PARAMS, "parameter count");

// One feature: log2(1 + x) / 32.
__device__ __forceinline__ float mlp_feat(double x) {
  return (float)(log2(1.0 + (x > 0 ? x : 0.0)) / 32.0);
}

// Selector input i of one iteration (0..7): n_f, m_f, n_u, m_u, largest
// frontier degree, V, E, and the unvisited-list size a pull step would need
// (V after a push, 0 after a pull), each log2(1 + x) / 32.  Eight threads
// compute the eight inputs side by side.
__device__ __forceinline__ float mlp_feature(int i, int64_t n_f, int64_t m_f, int64_t n_u,
                                             int64_t m_u, int64_t max_deg, int64_t V, int64_t E,
                                             int prev_pull) {
  int64_t x;
  switch (i) {
    case 0: x = n_f; break;
    case 1: x = m_f; break;
    case 2: x = n_u; break;
    case 3: x = m_u; break;
    case 4: x = max_deg; break;
    case 5: x = V; break;
    case 6: x = E; break;
    default: x = prev_pull ? 0 : V; break;
  }
  return mlp_feat((double)x);
}

// Forward pass on the features in s_x and argmin over the allowed actions
// (bit a of `allowed`).  Every thread of the workgroup must call it (it
// synchronises the workgroup); all of them get the same answer.  Every
// workgroup evaluates the same operations in the same order, so workgroups
// given equal inputs decide alike.
__device__ __forceinline__ int mlp_argmin(const float* __restrict__ params, const float* s_x,
                                          float* s_h1, float* s_h2, float* s_y, int allowed) {
  const int t = threadIdx.x;
  __syncthreads();
  if (t < kH) {
    float z = params[oB1 + t];
    for (int i = 0; i < kIn; ++i) z += params[oW1 + t * kIn + i] * s_x[i];
    s_h1[t] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  if (t < kH) {
    float z = params[oB2 + t];
    for (int i = 0; i < kH; ++i) z += params[oW2 + t * kH + i] * s_h1[i];
    s_h2[t] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  if (t < kOut) {
    float z = params[oB3 + t];
    for (int j = 0; j < kH; ++j) z += params[oW3 + t * kH + j] * s_h2[j];
    s_y[t] = z;
  }
  __syncthreads();
  int best = -1;
  for (int a = 0; a < kOut; ++a)
    if (((allowed >> a) & 1) && (best < 0 || s_y[a] < s_y[best])) best = a;
  return best;
}

}  // namespace gr
