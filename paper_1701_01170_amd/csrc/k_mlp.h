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

// The eight selector inputs of one iteration, written to s_x by the caller's
// thread: n_f, m_f, n_u, m_u, largest frontier degree, V, E, and the
// unvisited-list size a pull step would need (V after a push, 0 after a pull).
__device__ __forceinline__ void mlp_features(float* s_x, int64_t n_f, int64_t m_f, int64_t n_u,
                                             int64_t m_u, int64_t max_deg, int64_t V, int64_t E,
                                             int prev_pull) {
  s_x[0] = mlp_feat((double)n_f);
  s_x[1] = mlp_feat((double)m_f);
  s_x[2] = mlp_feat((double)n_u);
  s_x[3] = mlp_feat((double)m_u);
  s_x[4] = mlp_feat((double)max_deg);
  s_x[5] = mlp_feat((double)V);
  s_x[6] = mlp_feat((double)E);
  s_x[7] = mlp_feat(prev_pull ? 0.0 : (double)V);
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
