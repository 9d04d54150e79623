// Strategy-selector network: 8 inputs -> 32 -> 32 -> 4 outputs, ReLU on the
// hidden layers, fp32 (parameter layout in k_mlp.h).  The selector takes the
// argmin of the predicted step times over the actions the traversal allows.
//
// Kernels: batched forward; masked squared-error loss with its gradient
// (per-tile partial sums, then a fixed-order reduction: deterministic); Adam;
// and the fused inference kernel the traversal launches each iteration, which
// builds the eight features from the frontier statistics on the device.
#include "gr_internal.h"
#include "k_common.h"
#include "k_mlp.h"

namespace gr {

namespace {

constexpr int kTile = 64;  // samples per workgroup in the gradient kernel

__device__ __forceinline__ void load_params(const float* __restrict__ params, float* s_p) {
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) s_p[i] = params[i];
}

// Forward pass of one sample; h1/h2 receive the post-ReLU activations.
__device__ __forceinline__ void forward1(const float* p, const float* x, float* h1, float* h2,
                                         float* y) {
  for (int j = 0; j < kH; ++j) {
    float z = p[oB1 + j];
    for (int i = 0; i < kIn; ++i) z += p[oW1 + j * kIn + i] * x[i];
    h1[j] = z > 0.f ? z : 0.f;
  }
  for (int j = 0; j < kH; ++j) {
    float z = p[oB2 + j];
    for (int i = 0; i < kH; ++i) z += p[oW2 + j * kH + i] * h1[i];
    h2[j] = z > 0.f ? z : 0.f;
  }
  for (int o = 0; o < kOut; ++o) {
    float z = p[oB3 + o];
    for (int j = 0; j < kH; ++j) z += p[oW3 + o * kH + j] * h2[j];
    y[o] = z;
  }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params,
                                                     const float* __restrict__ X, int32_t n,
                                                     float* __restrict__ Y) {
  __shared__ float s_p[kNP];
  load_params(params, s_p);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kIn], h1[kH], h2[kH], y[kOut];
  for (int i = 0; i < kIn; ++i) x[i] = X[s * kIn + i];
  forward1(s_p, x, h1, h2, y);
  for (int o = 0; o < kOut; ++o) Y[s * kOut + o] = y[o];
}

// Per tile of 64 samples: forward and backward per sample (threads 0..63),
// then every parameter's contribution summed over the tile in sample order.
// partial[tile][kNP + 0] = sum of masked squared errors, [kNP + 1] = mask sum.
// The gradient of sum(M * (Y - T)^2) is accumulated here; the reduction
// divides by max(1, sum M).
__global__ __launch_bounds__(256) void k_mlp_grad_tiles(const float* __restrict__ params,
                                                        const float* __restrict__ X,
                                                        const float* __restrict__ T,
                                                        const float* __restrict__ M, int32_t n,
                                                        float* __restrict__ partial) {
  __shared__ float s_p[kNP];
  __shared__ float s_x[kTile][kIn];
  __shared__ float s_h1[kTile][kH];
  __shared__ float s_h2[kTile][kH];
  __shared__ float s_dz1[kTile][kH];
  __shared__ float s_dz2[kTile][kH];
  __shared__ float s_dy[kTile][kOut];
  __shared__ float s_l[kTile], s_m[kTile];
  load_params(params, s_p);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kTile) {
    const int64_t s = (int64_t)blockIdx.x * kTile + t;
    float x[kIn], h1[kH], h2[kH], y[kOut];
    float l = 0.f, msum = 0.f;
    if (s < n) {
      for (int i = 0; i < kIn; ++i) x[i] = X[s * kIn + i];
      forward1(s_p, x, h1, h2, y);
      float dy[kOut];
      for (int o = 0; o < kOut; ++o) {
        const float m = M[s * kOut + o];
        const float e = y[o] - T[s * kOut + o];
        dy[o] = 2.f * m * e;
        l += m * e * e;
        msum += m;
      }
      float dz2[kH];
      for (int j = 0; j < kH; ++j) {
        float g = 0.f;
        for (int o = 0; o < kOut; ++o) g += dy[o] * s_p[oW3 + o * kH + j];
        dz2[j] = h2[j] > 0.f ? g : 0.f;
      }
      for (int i = 0; i < kH; ++i) {
        float g = 0.f;
        for (int j = 0; j < kH; ++j) g += dz2[j] * s_p[oW2 + j * kH + i];
        s_dz1[t][i] = h1[i] > 0.f ? g : 0.f;
      }
      for (int i = 0; i < kIn; ++i) s_x[t][i] = x[i];
      for (int j = 0; j < kH; ++j) {
        s_h1[t][j] = h1[j];
        s_h2[t][j] = h2[j];
        s_dz2[t][j] = dz2[j];
      }
      for (int o = 0; o < kOut; ++o) s_dy[t][o] = dy[o];
    } else {
      for (int i = 0; i < kIn; ++i) s_x[t][i] = 0.f;
      for (int j = 0; j < kH; ++j) s_h1[t][j] = s_h2[t][j] = s_dz1[t][j] = s_dz2[t][j] = 0.f;
      for (int o = 0; o < kOut; ++o) s_dy[t][o] = 0.f;
    }
    s_l[t] = l;
    s_m[t] = msum;
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * (kNP + 2);
  for (int q = t; q < kNP; q += blockDim.x) {
    float acc = 0.f;
    if (q < oB1) {
      const int j = (q - oW1) / kIn, i = (q - oW1) % kIn;
      for (int s = 0; s < kTile; ++s) acc += s_dz1[s][j] * s_x[s][i];
    } else if (q < oW2) {
      const int j = q - oB1;
      for (int s = 0; s < kTile; ++s) acc += s_dz1[s][j];
    } else if (q < oB2) {
      const int j = (q - oW2) / kH, i = (q - oW2) % kH;
      for (int s = 0; s < kTile; ++s) acc += s_dz2[s][j] * s_h1[s][i];
    } else if (q < oW3) {
      const int j = q - oB2;
      for (int s = 0; s < kTile; ++s) acc += s_dz2[s][j];
    } else if (q < oB3) {
      const int o = (q - oW3) / kH, j = (q - oW3) % kH;
      for (int s = 0; s < kTile; ++s) acc += s_dy[s][o] * s_h2[s][j];
    } else {
      const int o = q - oB3;
      for (int s = 0; s < kTile; ++s) acc += s_dy[s][o];
    }
    out[q] = acc;
  }
  if (t == 0) {
    float l = 0.f, m = 0.f;
    for (int s = 0; s < kTile; ++s) {
      l += s_l[s];
      m += s_m[s];
    }
    out[kNP] = l;
    out[kNP + 1] = m;
  }
}

// Sum the tiles in tile order and scale by 1 / max(1, sum M).
__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float* __restrict__ partial,
                                                         int32_t n_tiles, float* __restrict__ grad,
                                                         float* __restrict__ loss) {
  __shared__ float s_den;
  if (threadIdx.x == 0) {
    float m = 0.f;
    for (int b = 0; b < n_tiles; ++b) m += partial[(int64_t)b * (kNP + 2) + kNP + 1];
    s_den = m > 1.f ? m : 1.f;
  }
  __syncthreads();
  const float inv = 1.f / s_den;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < kNP) {
    float acc = 0.f;
    for (int b = 0; b < n_tiles; ++b) acc += partial[(int64_t)b * (kNP + 2) + q];
    grad[q] = acc * inv;
  } else if (q == kNP && loss) {
    float acc = 0.f;
    for (int b = 0; b < n_tiles; ++b) acc += partial[(int64_t)b * (kNP + 2) + kNP];
    *loss = acc * inv;
  }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / c1) / (sqrt(v / c2) + eps) with c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// One wavefront: features of the current iteration (the frontier statistics
// of slot `sp` plus host-known totals), forward pass, argmin over the allowed
// actions (bit a of allowed) -> ctrl->action.  n_u_before / m_u_before are the
// unvisited counts before this frontier was visited (BFS), 0 for SSSP.
// Selector decision fused into the publication of the control block: the
// network runs first (its outputs go to the device control block and, taken
// from LDS, into the host copy), then every word is copied to host memory,
// ordered at system scope, and one thread releases the sequence number.
__global__ __launch_bounds__(128) void k_publish_select(MlpSelect m, Ctrl* __restrict__ ctrl,
                                                        uint32_t* __restrict__ dst, uint32_t* flag,
                                                        uint32_t seq, PublishExtra x) {
  __shared__ float s_p[kNP];
  __shared__ float s_x[kIn], s_h1[kH], s_h2[kH], s_y[kOut];
  __shared__ uint32_t s_dec[kOut + 1];
  // the parameters are staged in LDS with one coalesced burst: read layer by
  // layer from memory, each layer would wait for its own round trip
  for (int i = threadIdx.x; i < kNP; i += blockDim.x) s_p[i] = m.params[i];
  if (threadIdx.x < kIn) {
    const int64_t n_f = ctrl->n_f[m.sp], m_f = ctrl->m_f[m.sp];
    int64_t nub = m.n_u_before, mub = m.m_u_before;
    if (m.after_block) {
      const int k = ctrl->dl_levels;
      nub = m.V - ctrl->dl_vn[k & 1];
      mub = m.E - ctrl->dl_vm[k & 1];
    }
    int64_t n_u = nub > 0 ? nub - n_f : 0;
    int64_t m_u = mub > 0 ? mub - m_f : 0;
    if (m.ms_k > 0) {
      n_u = m.V - ctrl->ms_pairs / m.ms_k;
      m_u = m.E - ctrl->ms_pair_edges / m.ms_k;
    }
    // a batched traversal's last feature is its number of sources (its pull
    // builds no unvisited list, so the single-source meaning does not apply)
    s_x[threadIdx.x] = m.ms_k > 0 && threadIdx.x == kIn - 1
                           ? mlp_feat((double)m.ms_k)
                           : mlp_feature(threadIdx.x, n_f, m_f, n_u, m_u, ctrl->max_deg[m.sp], m.V,
                                         m.E, m.prev_pull);
  }
  const int best = mlp_argmin(s_p, s_x, s_h1, s_h2, s_y, m.allowed);
  if (threadIdx.x < kOut) {
    const float p = ((m.allowed >> threadIdx.x) & 1) ? s_y[threadIdx.x] : __builtin_inff();
    ctrl->pred[threadIdx.x] = p;
    s_dec[threadIdx.x] = __float_as_uint(p);
  }
  if (threadIdx.x == 0) {
    ctrl->action = best;
    s_dec[kOut] = (uint32_t)best;
  }
  __syncthreads();
  constexpr int kWords = (int)(sizeof(Ctrl) / 4);
  constexpr int kPred = (int)(offsetof(Ctrl, pred) / 4), kAction = (int)(offsetof(Ctrl, action) / 4);
  static_assert(offsetof(Ctrl, pred) % 4 == 0 && offsetof(Ctrl, action) % 4 == 0, "word offsets");
  const uint32_t* __restrict__ src = reinterpret_cast<const uint32_t*>(ctrl);
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) {
    uint32_t w;
    if (i >= kPred && i < kPred + kOut) w = s_dec[i - kPred];
    else if (i == kAction) w = s_dec[kOut];
    else w = src[i];
    dst[i] = w;
  }
  for (int i = threadIdx.x; i < x.n_words; i += blockDim.x) x.dst[i] = x.src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int mlp_tile() { return kTile; }

hipError_t launch_mlp_forward(const float* params, const float* X, int32_t n, float* Y,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_mlp_forward<<<blocks_for(n, 256), 256, 0, st>>>(params, X, n, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T,
                                const float* M, int32_t n, float* partial, float* grad,
                                float* loss, hipStream_t st) {
  const int tiles = (int)blocks_for(n > 0 ? n : 1, kTile);
  k_mlp_grad_tiles<<<tiles, 256, 0, st>>>(params, X, T, M, n, partial);
  k_mlp_grad_reduce<<<blocks_for(kNP + 1, 256), 256, 0, st>>>(partial, tiles, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st) {
  k_adam<<<blocks_for(n, 256), 256, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_publish_select(const MlpSelect& m, Ctrl* ctrl, Ctrl* host_dst,
                                 uint32_t* host_flag, uint32_t seq, hipStream_t st,
                                 const PublishExtra& extra) {
  static_assert(sizeof(Ctrl) % 4 == 0, "control block is copied as 32-bit words");
  k_publish_select<<<1, 128, 0, st>>>(m, ctrl, reinterpret_cast<uint32_t*>(host_dst), host_flag,
                                      seq, extra);
  return hipGetLastError();
}

}  // namespace gr
