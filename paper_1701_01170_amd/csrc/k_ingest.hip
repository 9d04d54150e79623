// Graph ingest kernels (CSR storage, Sec. 5.4): validation of device-side
// inputs, detection and sorting of adjacency lists that are not ascending
// (pull traversal and canonical parents rely on ascending neighbour order),
// degree / weight statistics, and the degree-ordered relabelling of the
// vertices (hubs first, so the per-vertex state the traversals touch most
// often shares few cache lines).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "gr_internal.h"
#include "k_common.h"

namespace gr {

namespace {

// flags_dev[0] bits: 1 = row_offsets[0] != 0, 2 = row_offsets[V] != E,
// 4 = row_offsets decreasing somewhere, 8 = a column index out of range.
__global__ __launch_bounds__(256) void k_csr_check(const int32_t* __restrict__ R,
                                                   const int32_t* __restrict__ C, int64_t V,
                                                   int64_t E, int64_t* __restrict__ flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t f = 0;
  if (i0 == 0) {
    if (R[0] != 0) f |= 1;
    if ((int64_t)R[V] != E) f |= 2;
  }
  for (int64_t v = i0; v < V; v += stride)
    if (R[v + 1] < R[v]) f |= 4;
  for (int64_t e = i0; e < E; e += stride) {
    int32_t c = C[e];
    if (c < 0 || (int64_t)c >= V) f |= 8;
  }
  if (f) atomicOr((unsigned long long*)flags, (unsigned long long)f);
}

__device__ __forceinline__ uint64_t sort_key(const int32_t* C, const uint32_t* W, int64_t e) {
  return ((uint64_t)(uint32_t)C[e] << 32) | (W ? (uint64_t)W[e] : 0ull);
}

// Rows whose (neighbour, weight) sequence is not non-decreasing: a lane
// checks a row of up to 64 entries, longer rows are checked by the whole
// wavefront, 64 adjacent pairs per step.
__global__ __launch_bounds__(256) void k_find_unsorted(const int32_t* __restrict__ R,
                                                       const int32_t* __restrict__ C,
                                                       const uint32_t* __restrict__ W, int64_t V,
                                                       int32_t* __restrict__ rows,
                                                       uint32_t* __restrict__ count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < V;
  int64_t rb = 0, re = 0;
  if (valid) {
    rb = R[v];
    re = R[v + 1];
  }
  bool bad = false;
  if (valid && re - rb <= kWave) {
    uint64_t prev = 0;
    for (int64_t e = rb; e < re; ++e) {
      const uint64_t k = sort_key(C, W, e);
      if (e > rb && k < prev) {
        bad = true;
        break;
      }
      prev = k;
    }
  }
  uint64_t big = __ballot(valid && re - rb > kWave);
  while (big) {
    const int l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const int64_t vb = __shfl(rb, l), ve = __shfl(re, l);
    bool any_bad = false;
    for (int64_t b = vb; b + 1 < ve && !any_bad; b += kWave) {
      const int64_t j = b + lane();
      const bool x = j + 1 < ve && sort_key(C, W, j + 1) < sort_key(C, W, j);
      any_bad = __any(x);
    }
    if (lane() == l) bad = any_bad;
  }
  uint32_t slot = wave_append(count, bad);
  if (bad) rows[slot] = (int32_t)v;
}

constexpr int kSortLds = 2048;

// One workgroup sorts one row with an all-ascending bitonic network
// (comparators i < l with l = i ^ (k-1) on the first step of each merge
// stage, i ^ j afterwards; positions at or beyond n act as +infinity).  Rows
// of up to kSortLds entries are sorted in LDS, longer ones in global scratch.
__global__ __launch_bounds__(256) void k_row_sort(const int32_t* __restrict__ R,
                                                  int32_t* __restrict__ C,
                                                  uint32_t* __restrict__ W,
                                                  const int32_t* __restrict__ rows,
                                                  uint64_t* __restrict__ scratch) {
  __shared__ uint64_t s_keys[kSortLds];
  const int32_t v = rows[blockIdx.x];
  const int64_t rb = R[v];
  const int64_t n = (int64_t)R[v + 1] - rb;
  uint64_t* keys = n <= kSortLds ? s_keys : scratch + rb;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) keys[i] = sort_key(C, W, rb + i);
  __syncthreads();
  int64_t N = 1;
  while (N < n) N <<= 1;
  for (int64_t k = 2; k <= N; k <<= 1) {
    for (int64_t j = k >> 1; j > 0; j >>= 1) {
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        int64_t l = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
        if (l > i && l < n) {
          uint64_t a = keys[i], b = keys[l];
          if (a > b) {
            keys[i] = b;
            keys[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    uint64_t k = keys[i];
    C[rb + i] = (int32_t)(k >> 32);
    if (W) W[rb + i] = (uint32_t)(k & 0xffffffffull);
  }
}

// out2[0] = max degree, out2[1] = max weight
__global__ __launch_bounds__(256) void k_graph_stats(const int32_t* __restrict__ R,
                                                     const uint32_t* __restrict__ W, int64_t V,
                                                     int64_t E, int64_t* __restrict__ out2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t md = 0, mw = 0;
  for (int64_t v = i0; v < V; v += stride) {
    int64_t d = (int64_t)R[v + 1] - R[v];
    md = d > md ? d : md;
  }
  if (W)
    for (int64_t e = i0; e < E; e += stride) {
      int64_t w = W[e];
      mw = w > mw ? w : mw;
    }
  md = wave_max(md);
  mw = wave_max(mw);
  if (lane() == 0) {
    atomicMax((unsigned long long*)&out2[0], (unsigned long long)md);
    atomicMax((unsigned long long*)&out2[1], (unsigned long long)mw);
  }
}

// Radix-sort keys for the degree order: descending degree; the stable sort
// keeps ascending ids among equal degrees.
__global__ __launch_bounds__(256) void k_degree_keys(const int32_t* __restrict__ R, int64_t V,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ ids) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) {
    keys[v] = ~(uint32_t)(R[v + 1] - R[v]);
    ids[v] = (int32_t)v;
  }
}

// perm: new id -> original id; inv: original id -> new id; deg_new[i] = the
// degree of new vertex i.
__global__ __launch_bounds__(256) void k_relabel_rows(const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ R, int64_t V,
                                                      int32_t* __restrict__ inv,
                                                      int32_t* __restrict__ deg_new) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V) {
    const int32_t v = perm[i];
    inv[v] = (int32_t)i;
    deg_new[i] = R[v + 1] - R[v];
  }
}

// One thread per relabelled edge: row i of the new CSR is row perm[i] of the
// old one with every neighbour renamed, in the old order (ascending original
// ids), weights alongside.
__global__ __launch_bounds__(256) void k_relabel_edges(
    const int32_t* __restrict__ R_new, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ inv, const int32_t* __restrict__ R, const int32_t* __restrict__ C,
    const uint32_t* __restrict__ W, int64_t V, int64_t E, int32_t* __restrict__ C_new,
    uint32_t* __restrict__ W_new) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
    const int i = upper_index(R_new, 0, (int)(V - 1), (int32_t)e);
    const int64_t src = (int64_t)R[perm[i]] + (e - R_new[i]);
    C_new[e] = inv[C[src]];
    if (W) W_new[e] = W[src];
  }
}

// The inverse: the CSR in original ids, from the relabelled one.
__global__ __launch_bounds__(256) void k_unrelabel_edges(
    const int32_t* __restrict__ R_orig, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ inv, const int32_t* __restrict__ R_new,
    const int32_t* __restrict__ C_new, const uint32_t* __restrict__ W_new, int64_t V, int64_t E,
    int32_t* __restrict__ C, uint32_t* __restrict__ W) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
    const int v = upper_index(R_orig, 0, (int)(V - 1), (int32_t)e);
    const int64_t src = (int64_t)R_new[inv[v]] + (e - R_orig[v]);
    C[e] = perm[C_new[src]];
    if (W) W[e] = W_new[src];
  }
}

inline unsigned capped_blocks(int64_t n, int per, unsigned cap) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

}  // namespace

hipError_t launch_csr_check(const int32_t* R, const int32_t* C, int64_t V, int64_t E,
                            int64_t* flags_dev, hipStream_t st) {
  k_csr_check<<<capped_blocks(V > E ? V : E, 256, 8192), 256, 0, st>>>(R, C, V, E, flags_dev);
  return hipGetLastError();
}

hipError_t launch_find_unsorted(const int32_t* R, const int32_t* C, const uint32_t* W, int64_t V,
                                int32_t* rows_out, uint32_t* count, hipStream_t st) {
  k_find_unsorted<<<capped_blocks(V, 256, 0x7fffffff), 256, 0, st>>>(R, C, W, V, rows_out, count);
  return hipGetLastError();
}

hipError_t launch_row_sort(int32_t* R, int32_t* C, uint32_t* W, int64_t V, const int32_t* rows,
                           int64_t n_rows, uint64_t* scratch, hipStream_t st) {
  (void)V;
  if (n_rows <= 0) return hipSuccess;
  k_row_sort<<<(unsigned)n_rows, 256, 0, st>>>(R, C, W, rows, scratch);
  return hipGetLastError();
}

hipError_t launch_graph_stats(const int32_t* R, const uint32_t* W, int64_t V, int64_t E,
                              int64_t* out2, hipStream_t st) {
  k_graph_stats<<<capped_blocks(V > E ? V : E, 256, 4096), 256, 0, st>>>(R, W, V, E, out2);
  return hipGetLastError();
}

hipError_t relabel_by_degree(const int32_t* R, const int32_t* C, const uint32_t* W, int64_t V,
                             int64_t E, int32_t* perm, int32_t* inv, int32_t* R_new,
                             int32_t* C_new, uint32_t* W_new, hipStream_t st) {
  uint32_t *keys = nullptr, *keys_out = nullptr;
  int32_t *ids = nullptr, *deg = nullptr;
  void* tmp = nullptr;
  size_t sort_bytes = 0, scan_bytes = 0;
  hipError_t e = hipSuccess;
  auto fin = [&](hipError_t r) {
    hipError_t s2 = hipStreamSynchronize(st);
    (void)hipFree(keys);
    (void)hipFree(keys_out);
    (void)hipFree(ids);
    (void)hipFree(deg);
    (void)hipFree(tmp);
    return r != hipSuccess ? r : s2;
  };
  if ((e = hipMalloc(&keys, sizeof(uint32_t) * V)) != hipSuccess) return fin(e);
  if ((e = hipMalloc(&keys_out, sizeof(uint32_t) * V)) != hipSuccess) return fin(e);
  if ((e = hipMalloc(&ids, sizeof(int32_t) * V)) != hipSuccess) return fin(e);
  if ((e = hipMalloc(&deg, sizeof(int32_t) * V)) != hipSuccess) return fin(e);
  if ((e = rocprim::radix_sort_pairs(nullptr, sort_bytes, keys, keys_out, ids, perm, (size_t)V, 0,
                                     32, st)) != hipSuccess)
    return fin(e);
  if ((e = rocprim::exclusive_scan(nullptr, scan_bytes, deg, R_new, 0, (size_t)V,
                                   rocprim::plus<int32_t>(), st)) != hipSuccess)
    return fin(e);
  if ((e = hipMalloc(&tmp, sort_bytes > scan_bytes ? sort_bytes : scan_bytes)) != hipSuccess)
    return fin(e);
  const unsigned gv = (unsigned)((V + 255) / 256);
  k_degree_keys<<<gv, 256, 0, st>>>(R, V, keys, ids);
  if ((e = rocprim::radix_sort_pairs(tmp, sort_bytes, keys, keys_out, ids, perm, (size_t)V, 0, 32,
                                     st)) != hipSuccess)
    return fin(e);
  k_relabel_rows<<<gv, 256, 0, st>>>(perm, R, V, inv, deg);
  if ((e = rocprim::exclusive_scan(tmp, scan_bytes, deg, R_new, 0, (size_t)V,
                                   rocprim::plus<int32_t>(), st)) != hipSuccess)
    return fin(e);
  if ((e = hipMemcpyAsync(R_new + V, R + V, sizeof(int32_t), hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return fin(e);
  if (E > 0)
    k_relabel_edges<<<capped_blocks(E, 256, 65536), 256, 0, st>>>(R_new, perm, inv, R, C, W, V, E,
                                                                  C_new, W_new);
  return fin(hipGetLastError());
}

hipError_t launch_unrelabel(const int32_t* R_orig, const int32_t* perm, const int32_t* inv,
                            const int32_t* R_new, const int32_t* C_new, const uint32_t* W_new,
                            int64_t V, int64_t E, int32_t* C, uint32_t* W, hipStream_t st) {
  if (E <= 0) return hipSuccess;
  k_unrelabel_edges<<<capped_blocks(E, 256, 65536), 256, 0, st>>>(R_orig, perm, inv, R_new, C_new,
                                                                  W_new, V, E, C, W);
  return hipGetLastError();
}

}  // namespace gr
