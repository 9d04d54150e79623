// Utility kernels: the HBM copy used to calibrate the bandwidth ceiling.
#include "gr_internal.h"
#include "k_common.h"

namespace gr {

namespace {

__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  k_copy16<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const uint4*>(src),
                                             static_cast<uint4*>(dst), n);
  return hipGetLastError();
}

}  // namespace gr
