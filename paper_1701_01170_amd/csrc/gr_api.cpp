// Host runtime of the gr_* C ABI: contexts, scratch pool, graph ingest and
// validation, and the enactors that drive the bulk-synchronous traversal loop
// (Sec. 3: a sequence of frontier-to-frontier steps until the frontier is
// empty; Alg. 1 for SSSP, Alg. 2 for direction-optimising BFS).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gr_internal.h"
#include "gr_policy.h"

namespace gr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

gr_status fail(gr_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// The static workspace of gr_bfs_static: one copy per device, held from the
// time the library's code is loaded on that device until the process ends.
// Host code never takes its address directly (in host code the name stands for
// a host-side shadow, not device memory); it uses the device address looked up
// with hipGetSymbolAddress, which ws_address keeps per device.
static __device__ __align__(256) char scratch[GR_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_ws_mutex;
void* g_ws_addr[kMaxDevices] = {};

// The device address of `device`'s workspace (the device must be current).
gr_status ws_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(GR_EUNSUPPORTED, "static workspace: device index " + std::to_string(device) +
                                     " beyond the library's table");
  std::lock_guard<std::mutex> lk(g_ws_mutex);
  if (!g_ws_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ws_addr[device] = p;
  }
  *out = g_ws_addr[device];
  return GR_OK;
}
}  // namespace

gr_status pool_get(gr_ctx* ctx, Slot s, size_t bytes, void** out) {
  DevBuf& b = ctx->pool[s];
  if (bytes == 0) bytes = 1;
  if (b.bytes < bytes) {
    if (b.ptr) {
      GR_HIP(hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t alloc = bytes + bytes / 8;  // head-room so slowly growing requests do not thrash
    hipError_t e = hipMalloc(&b.ptr, alloc);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      (void)hipGetLastError();
      return fail(GR_ENOMEM, "device allocation of " + std::to_string(alloc) + " bytes failed: " +
                                 hipGetErrorString(e));
    }
    b.bytes = alloc;
  }
  *out = b.ptr;
  return GR_OK;
}

namespace {

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline int64_t words_for(int64_t V) { return (V + 31) / 32; }

template <typename T>
gr_status pool_typed(gr_ctx* ctx, Slot s, size_t count, T** out) {
  void* p = nullptr;
  GR_TRY(pool_get(ctx, s, count * sizeof(T), &p));
  *out = static_cast<T*>(p);
  return GR_OK;
}

// Where a traversal takes its working arrays: the context's pool (grown on
// demand), or a fixed device region carved front to back in 256-byte aligned
// pieces (no allocation; asking for more than the region holds is GR_ERANGE).
// A slot asked for twice gets the same memory both times (a second request
// larger than the first is an error).  A measuring arena only adds up the
// bytes a fixed region would need and hands out null pointers.
struct Arena {
  gr_ctx* ctx = nullptr;
  char* base = nullptr;  // fixed region (null: the pool)
  size_t cap = 0;
  size_t used = 0;
  bool measure = false;
  bool taken[S_NSLOTS] = {};
  size_t off_of[S_NSLOTS] = {};
  size_t bytes_of[S_NSLOTS] = {};

  bool fixed() const { return base != nullptr || measure; }

  template <typename T>
  gr_status get(Slot s, size_t count, T** out) {
    if (!fixed()) return pool_typed(ctx, s, count, out);
    const size_t bytes = std::max<size_t>(count * sizeof(T), 1);
    if (!taken[s]) {
      const size_t off = (used + 255) / 256 * 256;
      if (!measure && off + bytes > cap)
        return fail(GR_ERANGE, "working arrays need more than the " + std::to_string(cap) +
                                   " bytes of the static device workspace");
      taken[s] = true;
      off_of[s] = off;
      bytes_of[s] = bytes;
      used = off + bytes;
    } else if (bytes > bytes_of[s]) {
      return fail(GR_ERANGE, "working array grew after the static workspace was laid out");
    }
    *out = measure ? nullptr : reinterpret_cast<T*>(base + off_of[s]);
    return GR_OK;
  }
};

// The control block after all work queued so far: a publishing kernel copies
// it to host memory and then bumps a sequence number, which the host polls;
// every 4096 polls the stream status is checked, so a failed launch or a
// faulted stream ends the wait with an error instead of a hang.
// With sel, the selector network decides on the device in the same kernel
// that publishes the control block.
// With pre, the degree scan of the frontier just measured is queued behind the
// publishing kernel, so it runs while the host waits and decides (the next
// load-balanced advance needs it; when the next step is something else it
// only used otherwise idle GPU time).
struct OffsetsJob {
  const int32_t* frontier;
  const uint32_t* n_f_dev;
  const int32_t* R;
  const int64_t* block_sums;
  const int64_t* total;
  int32_t* offsets;
  int32_t* rstart;
  int32_t* chunk_start;
  int32_t chunk;
};

gr_status read_ctrl(gr_ctx* ctx, Ctrl* dev, hipStream_t st, const MlpSelect* sel = nullptr,
                    const OffsetsJob* pre = nullptr, const PublishExtra* extra = nullptr) {
  const uint32_t seq = ++ctx->publish_seq;
  const PublishExtra x = extra ? *extra : PublishExtra{};
  if (sel)
    GR_HIP(launch_publish_select(*sel, dev, ctx->host_ctrl_dev, ctx->publish_flag_dev, seq, st, x));
  else
    GR_HIP(launch_publish(dev, ctx->host_ctrl_dev, ctx->publish_flag_dev, seq, st, x));
  if (pre)
    GR_HIP(launch_frontier_offsets(pre->frontier, 0, pre->R, pre->block_sums, pre->total,
                                   pre->offsets, pre->rstart, pre->chunk_start, pre->chunk, st,
                                   pre->n_f_dev));
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t i = 1;; ++i) {
    if (*ctx->publish_flag == seq) break;
    if ((i & 4095) == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipErrorNotReady) {
        if (std::chrono::steady_clock::now() - t0 > ctx->wait_limit)
          return fail(GR_EHIP, "the device did not publish the control block within " +
                                   std::to_string(ctx->wait_limit.count()) +
                                   " ms; the context's stream still holds unfinished work");
        continue;
      }
      if (e != hipSuccess) return fail(GR_EHIP, std::string("stream failed: ") + hipGetErrorString(e));
      if (*ctx->publish_flag != seq) return fail(GR_EHIP, "control block was not published");
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return GR_OK;
}

constexpr int kDefaultChunk = 8192;

// The push kernels' launch shape from the options (validated by check_opts).
AdvCfg adv_cfg(const gr_opts& o) {
  AdvCfg c;
  c.chunk = o.lb_chunk > 0 ? o.lb_chunk : kDefaultChunk;
  c.block = o.adv_block > 0 ? o.adv_block : 256;
  c.twc_wave_min = o.twc_wave_min > 0 ? o.twc_wave_min : -1;
  c.twc_block_min = o.twc_block_min > 0 ? o.twc_block_min : -1;
  return c;
}

}  // namespace
}  // namespace gr

using namespace gr;

// ============================================================================
// library, context
// ============================================================================

extern "C" int32_t gr_abi_version(void) { return GR_ABI_VERSION; }

extern "C" const char* gr_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t gr_abi_sizeof(int32_t which) {
  switch (which) {
    case 0: return (int32_t)sizeof(gr_opts);
    case 1: return (int32_t)sizeof(gr_run_stats);
    case 2: return (int32_t)sizeof(gr_level_trace);
    case 3: return (int32_t)sizeof(gr_graph_info);
    default: return -1;
  }
}

extern "C" void gr_opts_default(gr_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(gr_opts);
  o->policy = GR_POLICY_HEURISTIC;
  o->fixed_action = GR_PUSH_LB;
  o->lb_light_threshold = 4096;
  o->policy_seed = 0;
  o->do_a = 1.0f / 14.0f;
  o->do_b = 1.0f / 576.0f;
  o->lb_min_avg_degree = 5.0f;
  o->max_iterations = 0;
  o->lb_chunk = 0;
  o->trace_capacity = 0;
  o->trace = nullptr;
  o->trace_count = 0;
}

extern "C" gr_status gr_ctx_create(int32_t device, gr_ctx** out) {
  if (!out) return fail(GR_EINVAL, "gr_ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(GR_ENODEV, "no HIP device available");
  }
  if (device < 0 || device >= n)
    return fail(GR_ENODEV, "device " + std::to_string(device) + " out of range (" +
                               std::to_string(n) + " devices)");
  hipDeviceProp_t prop;
  GR_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GR_ENODEV, std::string("device is ") + prop.gcnArchName + ", the library is compiled for gfx950 only");
  DeviceGuard g(device);
  gr_ctx* c = new gr_ctx();
  c->device = device;
  c->cu_count = prop.multiProcessorCount;
  if (const char* w = std::getenv("GR_WAIT_LIMIT_MS")) {
    const long long ms = std::atoll(w);
    if (ms > 0) c->wait_limit = std::chrono::milliseconds(ms);
  }
  // control block mirror, block log and publish flag: coherent, device-mapped
  // pinned memory
  void* hc = nullptr;
  const size_t ctrl_bytes = (sizeof(Ctrl) + 255) / 256 * 256;
  const size_t dlog_bytes = (sizeof(int64_t) * 3 * kDlMaxLevels + 255) / 256 * 256;
  const size_t mirror_bytes = ctrl_bytes + dlog_bytes + 256;
  if (hipHostMalloc(&hc, mirror_bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete c;
    return fail(GR_ENOMEM, "pinned host allocation failed");
  }
  std::memset(hc, 0, mirror_bytes);
  void* hd = nullptr;
  if (hipHostGetDevicePointer(&hd, hc, 0) != hipSuccess) {
    (void)hipHostFree(hc);
    delete c;
    return fail(GR_EHIP, "hipHostGetDevicePointer failed");
  }
  if (gr_status ws = ws_address(device, &c->static_ws); ws != GR_OK) {
    (void)hipHostFree(hc);
    delete c;
    return ws;
  }
  c->host_ctrl = static_cast<Ctrl*>(hc);
  c->host_ctrl_dev = static_cast<Ctrl*>(hd);
  c->host_dlog = reinterpret_cast<int64_t*>(static_cast<char*>(hc) + ctrl_bytes);
  c->host_dlog_dev = reinterpret_cast<int64_t*>(static_cast<char*>(hd) + ctrl_bytes);
  const size_t flag_off = mirror_bytes - 256;
  c->publish_flag = reinterpret_cast<volatile uint32_t*>(static_cast<char*>(hc) + flag_off);
  c->publish_flag_dev = reinterpret_cast<uint32_t*>(static_cast<char*>(hd) + flag_off);
  if (hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_stop) != hipSuccess ||
      hipEventCreate(&c->ev_a) != hipSuccess || hipEventCreate(&c->ev_b) != hipSuccess ||
      hipEventCreate(&c->ev_k0) != hipSuccess || hipEventCreate(&c->ev_k1) != hipSuccess ||
      hipEventCreate(&c->ev_c0) != hipSuccess || hipEventCreate(&c->ev_c1) != hipSuccess) {
    gr_ctx_destroy(c);
    return fail(GR_EHIP, "hipEventCreate failed");
  }
  *out = c;
  return GR_OK;
}

extern "C" gr_status gr_ctx_destroy(gr_ctx* c) {
  if (!c) return GR_OK;
  DeviceGuard g(c->device);
  for (auto& b : c->pool)
    if (b.ptr) (void)hipFree(b.ptr);
  if (c->host_ctrl) (void)hipHostFree(c->host_ctrl);
  for (auto& kv : c->block_graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t ev : {c->ev_start, c->ev_stop, c->ev_a, c->ev_b, c->ev_k0, c->ev_k1, c->ev_c0,
                        c->ev_c1})
    if (ev) (void)hipEventDestroy(ev);
  delete c;
  return GR_OK;
}

// ============================================================================
// graphs
// ============================================================================

extern "C" gr_status gr_validate_csr(int64_t V, int64_t E, const int32_t* R, const int32_t* C) {
  if (V < 1 || V > (int64_t)INT32_MAX - 1)
    return fail(GR_ERANGE, "n_vertices must be in [1, 2^31 - 2], got " + std::to_string(V));
  if (E < 0 || E > (int64_t)INT32_MAX)
    return fail(GR_ERANGE, "n_edges must be in [0, 2^31 - 1], got " + std::to_string(E));
  if (!R) return fail(GR_EINVAL, "row_offsets is NULL");
  if (E > 0 && !C) return fail(GR_EINVAL, "col_indices is NULL");
  if (R[0] != 0) return fail(GR_EINVAL, "row_offsets[0] must be 0");
  for (int64_t v = 0; v < V; ++v)
    if (R[v + 1] < R[v])
      return fail(GR_EINVAL, "row_offsets decreases at vertex " + std::to_string(v));
  if ((int64_t)R[V] != E)
    return fail(GR_EINVAL, "row_offsets[V] = " + std::to_string(R[V]) + " != n_edges = " +
                               std::to_string(E));
  for (int64_t e = 0; e < E; ++e)
    if (C[e] < 0 || (int64_t)C[e] >= V)
      return fail(GR_EINVAL, "col_indices[" + std::to_string(e) + "] = " + std::to_string(C[e]) +
                                 " out of range");
  return GR_OK;
}

namespace {

void free_graph_buffers(gr_graph* g) {
  if (g->R) (void)hipFree(g->R);
  if (g->C) (void)hipFree(g->C);
  if (g->W) (void)hipFree(g->W);
  if (g->perm) (void)hipFree(g->perm);
  if (g->inv) (void)hipFree(g->inv);
  if (g->R_orig) (void)hipFree(g->R_orig);
  g->R = nullptr;
  g->C = nullptr;
  g->W = nullptr;
  g->perm = nullptr;
  g->inv = nullptr;
  g->R_orig = nullptr;
  g->inv_host.clear();
}

gr_status ingest(gr_ctx* ctx, gr_graph* g, const int32_t* R, const int32_t* C, const uint32_t* W,
                 bool device_input, hipStream_t st) {
  const int64_t V = g->V, E = g->E;
  const hipMemcpyKind kind = device_input ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  GR_HIP(hipMalloc(&g->R, sizeof(int32_t) * (V + 1)));
  GR_HIP(hipMalloc(&g->C, sizeof(int32_t) * std::max<int64_t>(E, 1)));
  if (W) GR_HIP(hipMalloc(&g->W, sizeof(uint32_t) * std::max<int64_t>(E, 1)));
  GR_HIP(hipMemcpyAsync(g->R, R, sizeof(int32_t) * (V + 1), kind, st));
  if (E > 0) GR_HIP(hipMemcpyAsync(g->C, C, sizeof(int32_t) * E, kind, st));
  if (W && E > 0) GR_HIP(hipMemcpyAsync(g->W, W, sizeof(uint32_t) * E, kind, st));

  // small scratch: [0] csr flags, [1] max degree, [2] max weight, [3] unsorted count
  int64_t* tmp = nullptr;
  GR_HIP(hipMalloc(&tmp, sizeof(int64_t) * 4));
  struct TmpFree {
    int64_t* p;
    ~TmpFree() { (void)hipFree(p); }
  } tf{tmp};
  GR_HIP(hipMemsetAsync(tmp, 0, sizeof(int64_t) * 4, st));
  int64_t host4[4] = {0, 0, 0, 0};
  if (device_input) {
    GR_HIP(launch_csr_check(g->R, g->C, V, E, tmp, st));
    GR_HIP(hipMemcpyAsync(host4, tmp, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    GR_HIP(hipStreamSynchronize(st));
    if (host4[0]) {
      std::string why;
      if (host4[0] & 1) why += " row_offsets[0] != 0;";
      if (host4[0] & 2) why += " row_offsets[V] != n_edges;";
      if (host4[0] & 4) why += " row_offsets decreasing;";
      if (host4[0] & 8) why += " col_indices out of range;";
      return fail(GR_EINVAL, "malformed device CSR:" + why);
    }
  }
  // adjacency lists must be ascending (pull traversal, canonical parents)
  int32_t* rows = nullptr;
  GR_HIP(hipMalloc(&rows, sizeof(int32_t) * V));
  struct RowsFree {
    int32_t* p;
    ~RowsFree() { (void)hipFree(p); }
  } rf{rows};
  uint32_t* ucount = reinterpret_cast<uint32_t*>(tmp + 3);
  GR_HIP(launch_find_unsorted(g->R, g->C, g->W, V, rows, ucount, st));
  GR_HIP(hipMemcpyAsync(&host4[3], tmp + 3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  GR_HIP(hipStreamSynchronize(st));
  const int64_t n_unsorted = (int64_t)(uint32_t)(host4[3] & 0xffffffff);
  if (n_unsorted > 0) {
    uint64_t* scratch = nullptr;
    GR_HIP(hipMalloc(&scratch, sizeof(uint64_t) * std::max<int64_t>(E, 1)));
    hipError_t e1 = launch_row_sort(g->R, g->C, g->W, V, rows, n_unsorted, scratch, st);
    hipError_t e2 = hipStreamSynchronize(st);
    (void)hipFree(scratch);
    GR_HIP(e1);
    GR_HIP(e2);
    g->resorted = 1;
  }
  GR_HIP(launch_graph_stats(g->R, g->W, V, E, tmp + 1, st));
  GR_HIP(hipMemcpyAsync(&host4[1], tmp + 1, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  GR_HIP(hipStreamSynchronize(st));
  g->max_degree = host4[1];
  g->max_weight = (uint32_t)host4[2];
  (void)ctx;
  if (!(g->flags & GR_RENUMBER)) return GR_OK;
  // renumber by descending degree (see gr_graph)
  int32_t *perm = nullptr, *inv = nullptr, *R_new = nullptr, *C_new = nullptr;
  uint32_t* W_new = nullptr;
  auto undo = [&]() {
    (void)hipFree(perm);
    (void)hipFree(inv);
    (void)hipFree(R_new);
    (void)hipFree(C_new);
    (void)hipFree(W_new);
  };
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&perm, sizeof(int32_t) * V)) == hipSuccess &&
      (e = hipMalloc(&inv, sizeof(int32_t) * V)) == hipSuccess &&
      (e = hipMalloc(&R_new, sizeof(int32_t) * (V + 1))) == hipSuccess &&
      (e = hipMalloc(&C_new, sizeof(int32_t) * std::max<int64_t>(E, 1))) == hipSuccess &&
      (!g->W || (e = hipMalloc(&W_new, sizeof(uint32_t) * std::max<int64_t>(E, 1))) == hipSuccess))
    e = relabel_by_degree(g->R, g->C, g->W, V, E, perm, inv, R_new, C_new, W_new, st);
  if (e != hipSuccess) {
    undo();
    return fail(e == hipErrorOutOfMemory ? GR_ENOMEM : GR_EHIP,
                std::string("vertex renumbering: ") + hipGetErrorString(e));
  }
  g->inv_host.resize((size_t)V);
  e = hipMemcpy(g->inv_host.data(), inv, sizeof(int32_t) * V, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    undo();
    return fail(GR_EHIP, std::string("vertex renumbering: ") + hipGetErrorString(e));
  }
  (void)hipFree(g->C);
  if (g->W) (void)hipFree(g->W);
  g->R_orig = g->R;
  g->R = R_new;
  g->C = C_new;
  g->W = W_new;
  g->perm = perm;
  g->inv = inv;
  return GR_OK;
}

}  // namespace

extern "C" gr_status gr_graph_from_csr(gr_ctx* ctx, int64_t V, int64_t E, const int32_t* R,
                                       const int32_t* C, const uint32_t* W, uint32_t flags,
                                       void* stream, gr_graph** out) {
  if (!out) return fail(GR_EINVAL, "gr_graph_from_csr: out is NULL");
  *out = nullptr;
  if (flags & ~(GR_SYMMETRIC | GR_DEVICE_INPUT | GR_RENUMBER))
    return fail(GR_EINVAL, "unknown flags");
  const bool device_input = (flags & GR_DEVICE_INPUT) != 0;
  if (device_input) {
    if (V < 1 || V > (int64_t)INT32_MAX - 1)
      return fail(GR_ERANGE, "n_vertices must be in [1, 2^31 - 2], got " + std::to_string(V));
    if (E < 0 || E > (int64_t)INT32_MAX)
      return fail(GR_ERANGE, "n_edges must be in [0, 2^31 - 1], got " + std::to_string(E));
    if (!R || (E > 0 && !C)) return fail(GR_EINVAL, "CSR pointer is NULL");
  } else {
    GR_TRY(gr_validate_csr(V, E, R, C));
  }
  if (!ctx) return fail(GR_EINVAL, "ctx is NULL");
  DeviceGuard dg(ctx->device);
  gr_graph* g = new gr_graph();
  g->ctx = ctx;
  g->V = V;
  g->E = E;
  g->flags = flags;
  gr_status s = ingest(ctx, g, R, C, W, device_input, static_cast<hipStream_t>(stream));
  if (s != GR_OK) {
    free_graph_buffers(g);
    delete g;
    return s;
  }
  *out = g;
  return GR_OK;
}

extern "C" gr_status gr_graph_free(gr_graph* g) {
  if (!g) return GR_OK;
  DeviceGuard dg(g->ctx->device);
  free_graph_buffers(g);
  delete g;
  return GR_OK;
}

extern "C" gr_status gr_graph_get_info(const gr_graph* g, gr_graph_info* out) {
  if (!g || !out) return fail(GR_EINVAL, "gr_graph_get_info: NULL argument");
  out->n_vertices = g->V;
  out->n_edges = g->E;
  out->max_degree = g->max_degree;
  out->flags = g->flags;
  out->weighted = g->W != nullptr;
  out->max_weight = g->max_weight;
  out->resorted = g->resorted;
  return GR_OK;
}

extern "C" gr_status gr_graph_export(const gr_graph* g, int32_t* R, int32_t* C, uint32_t* W,
                                     void* stream) {
  if (!g || !R || (g->E > 0 && !C)) return fail(GR_EINVAL, "gr_graph_export: NULL argument");
  if (W && !g->W) return fail(GR_EINVAL, "graph has no weights");
  DeviceGuard dg(g->ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (g->perm) {
    GR_HIP(hipMemcpyAsync(R, g->R_orig, sizeof(int32_t) * (g->V + 1), hipMemcpyDeviceToDevice, st));
    GR_HIP(launch_unrelabel(g->R_orig, g->perm, g->inv, g->R, g->C, W ? g->W : nullptr, g->V, g->E,
                            C, W, st));
  } else {
    GR_HIP(hipMemcpyAsync(R, g->R, sizeof(int32_t) * (g->V + 1), hipMemcpyDeviceToDevice, st));
    if (g->E > 0) {
      GR_HIP(hipMemcpyAsync(C, g->C, sizeof(int32_t) * g->E, hipMemcpyDeviceToDevice, st));
      if (W) GR_HIP(hipMemcpyAsync(W, g->W, sizeof(uint32_t) * g->E, hipMemcpyDeviceToDevice, st));
    }
  }
  GR_HIP(hipStreamSynchronize(st));
  return GR_OK;
}

// ============================================================================
// traversal helpers
// ============================================================================

namespace {

gr_status check_opts(gr_opts* opts, gr_opts* local) {
  if (!opts) {
    gr_opts_default(local);
    return GR_OK;
  }
  if (opts->struct_size != sizeof(gr_opts))
    return fail(GR_EINVAL, "opts->struct_size mismatch (call gr_opts_default)");
  if (opts->policy < GR_POLICY_HEURISTIC || opts->policy > GR_POLICY_RANDOM)
    return fail(GR_EINVAL, "opts->policy out of range");
  if (opts->fixed_action < GR_PUSH_TWC || opts->fixed_action > GR_PULL_LB)
    return fail(GR_EINVAL, "opts->fixed_action out of range");
  if (!(opts->do_a >= 0.0f) || !(opts->do_b >= 0.0f)) return fail(GR_EINVAL, "do_a/do_b must be >= 0");
  if (opts->lb_chunk != 0 && opts->lb_chunk != 512 && opts->lb_chunk != 1024 &&
      opts->lb_chunk != 2048 && opts->lb_chunk != 4096 &&
      opts->lb_chunk != 8192 && opts->lb_chunk != 16384)
    return fail(GR_EINVAL, "opts->lb_chunk must be 0 (default), 512, 1024, 2048, 4096, 8192 or 16384");
  if (opts->trace_capacity < 0 || (opts->trace_capacity > 0 && !opts->trace))
    return fail(GR_EINVAL, "opts->trace is NULL with a positive capacity");
  if (opts->device_max_edges > (1 << 24))
    return fail(GR_EINVAL, "opts->device_max_edges must be at most 1 << 24");
  if (opts->sssp_delta < 0) return fail(GR_EINVAL, "opts->sssp_delta must be >= 0");
  if (!(opts->learned_margin >= 0.0f) || !std::isfinite(opts->learned_margin))
    return fail(GR_EINVAL, "opts->learned_margin must be finite and >= 0");
  if (opts->adv_block != 0 && opts->adv_block != 128 && opts->adv_block != 256 &&
      opts->adv_block != 512)
    return fail(GR_EINVAL, "opts->adv_block must be 0 (default 256), 128, 256 or 512");
  if (opts->twc_wave_min < 0 || opts->twc_block_min < 0)
    return fail(GR_EINVAL, "opts->twc_wave_min / twc_block_min must be >= 0");
  if (opts->twc_wave_min > 0 && opts->twc_block_min > 0 && opts->twc_block_min < opts->twc_wave_min)
    return fail(GR_EINVAL, "opts->twc_block_min must be >= twc_wave_min");
  if (opts->graph_blocks != 0 && opts->graph_blocks != 1)
    return fail(GR_EINVAL, "opts->graph_blocks must be 0 or 1");
  if (opts->sssp_opt_off & ~(GR_SSSP_OPT_CULL | GR_SSSP_OPT_BINS))
    return fail(GR_EINVAL, "opts->sssp_opt_off: unknown bits");
  if (opts->sssp_multi_sweep != 0 && opts->sssp_multi_sweep != 1)
    return fail(GR_EINVAL, "opts->sssp_multi_sweep must be 0 or 1");
  if (opts->trace_steps_off != 0 && opts->trace_steps_off != 1)
    return fail(GR_EINVAL, "opts->trace_steps_off must be 0 or 1");
  if (opts->bc_dir < 0 || opts->bc_dir > 15 || (opts->bc_dir & 3) == 3 || (opts->bc_dir >> 2) == 3)
    return fail(GR_EINVAL, "opts->bc_dir: each pass takes GR_BC_DIR_AUTO, _PUSH or _PULL");
  if (opts->bfs_filter < GR_BFS_FILTER_AUTO || opts->bfs_filter > GR_BFS_FILTER_IDEMPOTENT)
    return fail(GR_EINVAL, "opts->bfs_filter out of range");
  if (opts->idem_culls_off & ~(int32_t)(GR_IDEM_CULL_WAVE | GR_IDEM_CULL_HISTORY | GR_IDEM_CULL_LABEL))
    return fail(GR_EINVAL, "opts->idem_culls_off has unknown bits");
  if (opts->idem_table_log2 != 0 && opts->idem_table_log2 != 8 && opts->idem_table_log2 != 10 &&
      opts->idem_table_log2 != 12)
    return fail(GR_EINVAL, "opts->idem_table_log2 must be 0 (default 10), 8, 10 or 12");
  *local = *opts;
  return GR_OK;
}

// Milliseconds between two recorded events.  The host can observe a
// published control block before the runtime has retired events recorded
// ahead of it, so wait for the later event first.
gr_status elapsed_ms(hipEvent_t a, hipEvent_t b, float* ms) {
  GR_HIP(hipEventSynchronize(b));
  GR_HIP(hipEventElapsedTime(ms, a, b));
  return GR_OK;
}

// Trace record of one iteration with the given step and kernel times.
// Work of one iteration's advance, for its trace record: input vertices read
// (push: the frontier; pull: the unvisited vertices or list entries scanned)
// and edges read (push: m_f; pull: neighbours scanned).
struct StepWork {
  int64_t n_in;
  int64_t inspected;
  int64_t n_cand = -1;  // entries before the exact filter (< 0: the filter was exact, n_next)
};

gr_status record_trace_times(gr_opts* opts, const LevelFeatures& lf, int action, int kernel,
                             int64_t n_next, float step_ms, float kernel_ms, StepWork w) {
  if (!opts || !opts->trace) return GR_OK;
  int i = opts->trace_count++;
  if (i >= opts->trace_capacity) return GR_OK;
  gr_level_trace& t = opts->trace[i];
  t.level = lf.level;
  t.action = action;
  t.n_f = lf.n_f;
  t.m_f = lf.m_f;
  t.n_u = lf.n_u;
  t.m_u = lf.m_u;
  t.max_deg_f = lf.max_deg_f;
  selector_features(lf, t.features);
  t.step_us = step_ms * 1000.0f;
  t.kernel_us = kernel_ms * 1000.0f;
  t.kernel = kernel;
  t.n_next = n_next;
  t.n_in = w.n_in;
  t.inspected = w.inspected;
  t.n_cand = w.n_cand >= 0 ? w.n_cand : n_next;
  return GR_OK;
}

// Event-timed record of one iteration: ev_a..ev_b brackets the whole step
// (not recorded with trace_steps_off), ev_k0..ev_k1 the advance kernel alone.
gr_status record_trace(gr_ctx* ctx, gr_opts* opts, const LevelFeatures& lf, int action,
                       int kernel, int64_t n_next, StepWork w) {
  if (!opts || !opts->trace || opts->trace_count >= opts->trace_capacity) {
    if (opts && opts->trace) opts->trace_count++;
    return GR_OK;
  }
  float step_ms = 0.f, kernel_ms = 0.f;
  if (!opts->trace_steps_off) GR_TRY(elapsed_ms(ctx->ev_a, ctx->ev_b, &step_ms));
  GR_TRY(elapsed_ms(ctx->ev_k0, ctx->ev_k1, &kernel_ms));
  return record_trace_times(opts, lf, action, kernel, n_next, step_ms, kernel_ms, w);
}

// ---- iteration control: device-predicated blocks of push levels ----------
constexpr int kDlFirstLen = 4;              // levels in the first block (then adapted per block)
constexpr int64_t kDlDefaultMaxEdges = 1 << 18;
constexpr int kTraceKernelDstep = 6;
constexpr int kTraceKernelRefill = 7;
constexpr int kTraceKernelPullList = 11;
constexpr int kTraceKernelIdem = 12;  // idempotent BFS push: 12 + (0 TWC, 1 LB_LIGHT, 2 LB)
constexpr int kTraceMarksOffset = 8;  // SSSP relaxation with the byte-mark filter: 8 + (0 TWC, 1 LB_LIGHT, 2 LB)
// SSSP iterations whose frontier has at least V / kSsspMarksDivisor edges use
// the byte-mark filter (and with it the cull and the distance bins of its
// compaction).  R-MAT 22, mean SSSP over 12 sources: 2.25 ms from V / 4,
// 2.21 ms from V / 8, 2.16-2.20 ms from V / 16, 2.19 ms from V / 32.
constexpr int64_t kSsspMarksDivisor = 16;
// ... and screen their edges with the one-byte distance mirror once the
// frontiers so far, this one included, and the far pile of the priority queue
// sum to at least V / kSsspMirrorDivisor vertices (an estimate of the vertices
// reached): before that most edges reach unvisited vertices, pass the screen
// anyway and pay for both gathers.  With the cull of vertices already relaxed
// with their final distance and the distance-binned frontier, R-MAT 22 SSSP
// measured 2.57-2.59 ms with the screen from V / 8, 2.61-2.65 ms from V / 2,
// 2.76 ms from V and 2.77 ms without it.
constexpr int64_t kSsspMirrorDivisor = 8;

struct DlPlan {
  bool on = false;
  int64_t max_m = 0;
  double do_a = -1.0;   // device push -> pull test (< 0: none)

  int len = kDlFirstLen;
  int blocks = 256;
  int64_t* log = nullptr;
  bool graph = false;   // record each block as a hipGraph
};
constexpr int kGraphKeyBfs = 0, kGraphKeySssp = 1, kGraphKeySsspPq = 2;

// hipGraph iteration control.  While a block of device-predicated levels is
// enqueued, its launches go to the context's capture stream (nothing runs
// there); the graph is then instantiated -- or, when a block of the same shape
// ran before, the kept instance is updated with the new arguments -- and
// launched on the caller's stream.  The guard ends a capture that an error
// left open.
struct BlockCapture {
  gr_ctx* ctx = nullptr;
  bool active = false;
  ~BlockCapture() {
    if (!active) return;
    hipGraph_t gph = nullptr;
    (void)hipStreamEndCapture(ctx->cap_stream, &gph);
    if (gph) (void)hipGraphDestroy(gph);
    (void)hipGetLastError();
  }
};

gr_status block_capture_begin(gr_ctx* ctx, BlockCapture* bc, hipStream_t* enqueue_on) {
  if (!ctx->cap_stream) GR_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  GR_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  bc->ctx = ctx;
  bc->active = true;
  *enqueue_on = ctx->cap_stream;
  return GR_OK;
}

gr_status block_capture_launch(gr_ctx* ctx, BlockCapture* bc, int key, hipStream_t st) {
  hipGraph_t gph = nullptr;
  bc->active = false;
  GR_HIP(hipStreamEndCapture(ctx->cap_stream, &gph));
  struct GraphFree {
    hipGraph_t g;
    ~GraphFree() {
      if (g) (void)hipGraphDestroy(g);
    }
  } gf{gph};
  auto it = ctx->block_graphs.find(key);
  bool updated = false;
  if (it != ctx->block_graphs.end()) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
    if (hipGraphExecUpdate(it->second, gph, &err_node, &res) == hipSuccess &&
        res == hipGraphExecUpdateSuccess) {
      updated = true;
    } else {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(it->second);
      ctx->block_graphs.erase(it);
    }
  }
  if (!updated) {
    hipGraphExec_t exec = nullptr;
    GR_HIP(hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0));
    ctx->block_graphs[key] = exec;
  }
  GR_HIP(hipGraphLaunch(ctx->block_graphs[key], st));
  return GR_OK;
}

gr_status dl_plan(gr_ctx* ctx, Arena& ar, const gr_opts& o, bool pull_ok, bool learned,
                  bool tracing, DlPlan* d) {
  const bool heuristic = o.policy == GR_POLICY_HEURISTIC ||
                         (o.policy == GR_POLICY_LEARNED && !learned);
  d->on = o.device_max_edges >= 0 && (heuristic || learned || o.policy == GR_POLICY_FIXED);
  d->max_m = o.device_max_edges > 0 ? o.device_max_edges : kDlDefaultMaxEdges;
  d->do_a = (heuristic || learned) && pull_ok ? (double)o.do_a : -1.0;

  d->len = kDlFirstLen;
  d->blocks = ctx->cu_count > 0 ? ctx->cu_count : 256;
  d->log = nullptr;
  d->graph = o.graph_blocks == 1 && !tracing && !ar.fixed();
  if (d->on && tracing) GR_TRY(ar.get(S_DLOG, 3 * kDlMaxLevels, &d->log));
  return GR_OK;
}

}  // namespace

// ============================================================================
// BFS enactor (Sec. 6.1, Alg. 2)
// ============================================================================

namespace {
// Push steps on symmetric graphs find parents either with an atomic min during
// the expansion (cheap while the frontier has few edges) or with the
// ascending-scan fix-up afterwards (cheap once the frontier is large: the first
// frontier neighbour is found early).  Both give the smallest-id parent.
constexpr int64_t kAtomicParentMaxEdges = 1 << 20;
// Push levels whose frontier has at least V / kMarksFilterDivisor edges use the
// non-atomic filter (byte marks + one ordered compaction pass over all V);
// smaller ones cull with atomics on the visited bitmap.
constexpr int64_t kMarksFilterDivisor = 4;
// A pull level reads the unvisited list the previous pull level left when it
// has at most V / kPullListDivisor entries; a longer list is slower to scan
// lane by lane than the bitmap (whose runs probe first neighbours together).
constexpr int64_t kPullListDivisor = 16;

// The byte-mark buffer is all zero between uses (the compaction clears what it
// reads); a fresh allocation is cleared once here.  A fixed arena's marks are
// cleared at the start of every call instead (see bfs_run), since the region
// keeps whatever an earlier call, possibly a failed one, left there.
gr_status marks_buffer(gr_ctx* ctx, Arena& ar, int64_t V, uint8_t** out, hipStream_t st) {
  const size_t bytes = (size_t)((V + 31) / 32) * 32;
  if (ar.fixed()) return ar.get(S_MARKS, bytes, out);
  const bool fresh = ctx->pool[S_MARKS].bytes < bytes;
  void* p = nullptr;
  GR_TRY(pool_get(ctx, S_MARKS, bytes, &p));
  if (fresh) GR_HIP(launch_fill_u32(static_cast<uint32_t*>(p), (int64_t)(ctx->pool[S_MARKS].bytes / 4),
                                    0u, st));
  *out = static_cast<uint8_t*>(p);
  return GR_OK;
}
}  // namespace

namespace {
gr_status bfs_check(const char* who, gr_ctx* ctx, const gr_graph* g, int32_t source,
                    const int32_t* depth) {
  const std::string w(who);
  if (!ctx || !g) return fail(GR_EINVAL, w + ": ctx or graph is NULL");
  if (g->ctx != ctx) return fail(GR_EINVAL, w + ": graph belongs to another context");
  if (!depth) return fail(GR_EINVAL, w + ": depth is NULL");
  if (source < 0 || (int64_t)source >= g->V)
    return fail(GR_EINVAL, w + ": source " + std::to_string(source) + " out of range");
  return GR_OK;
}

// The BFS working arrays.  In a fixed arena every one of them is laid out
// here, up front, so that measuring this layout gives the bytes a call needs;
// the pool hands out the byte marks lazily (marks_buffer).
struct BfsArrays {
  uint32_t* bm = nullptr;
  int32_t *qA = nullptr, *qB = nullptr, *qC = nullptr;
  int32_t *offsets = nullptr, *rstart = nullptr, *chunks = nullptr;
  int64_t* bsums = nullptr;
  Ctrl* ctrl = nullptr;
  uint8_t* marks = nullptr;            // fixed arenas only
  int32_t *depth = nullptr, *parent = nullptr;  // renumbered graphs only
  int32_t *ul0 = nullptr, *ul1 = nullptr;       // symmetric graphs only
  int64_t* dlog = nullptr;             // fixed arenas, traced calls only
  int32_t* cand = nullptr;             // idempotent advance only
};

gr_status bfs_layout(Arena& ar, int64_t V, int64_t E, bool pull_ok, bool renumbered,
                     bool want_parent, bool tracing, bool idem, BfsArrays* a) {
  GR_TRY(ar.get(S_BM, 2 * words_for(V), &a->bm));
  GR_TRY(ar.get(S_Q_A, V, &a->qA));
  GR_TRY(ar.get(S_Q_B, V, &a->qB));
  GR_TRY(ar.get(S_Q_C, V, &a->qC));
  GR_TRY(ar.get(S_OFFSETS, V + 1, &a->offsets));
  GR_TRY(ar.get(S_RSTART, V, &a->rstart));
  GR_TRY(ar.get(S_CHUNKS, E / 512 + 2, &a->chunks));
  GR_TRY(ar.get(S_BLOCK_SUMS, stats_grid() + 1, &a->bsums));
  GR_TRY(ar.get(S_CTRL, 1, &a->ctrl));
  if (ar.fixed()) GR_TRY(ar.get(S_MARKS, (size_t)((V + 31) / 32) * 32, &a->marks));
  if (renumbered) {
    GR_TRY(ar.get(S_DEPTH, V, &a->depth));
    if (want_parent) GR_TRY(ar.get(S_PARENT, V, &a->parent));
  }
  if (pull_ok) {
    GR_TRY(ar.get(S_UL_A, V, &a->ul0));
    GR_TRY(ar.get(S_UL_B, V, &a->ul1));
  }
  if (ar.fixed() && tracing) GR_TRY(ar.get(S_DLOG, 3 * kDlMaxLevels, &a->dlog));
  if (idem) GR_TRY(ar.get(S_CAND, V, &a->cand));
  return GR_OK;
}

// The idempotent advance needs the parent fix-up, which scans out-edges as
// in-edges: symmetric graphs only.
bool bfs_idem_on(const gr_opts& o, bool pull_ok) {
  return o.bfs_filter == GR_BFS_FILTER_IDEMPOTENT && pull_ok;
}

// The BFS enactor; its working arrays come from `ar` (arguments checked by
// the caller, device current).
gr_status bfs_run(gr_ctx* ctx, const gr_graph* g, int32_t source, int32_t* depth, int32_t* parent,
                  gr_opts* opts_in, const gr_opts& opts, hipStream_t st, gr_run_stats* stats,
                  Arena& ar, bool internal_ids = false) {
  const int64_t V = g->V, E = g->E, NW = words_for(V);
  const bool pull_ok = (g->flags & GR_SYMMETRIC) != 0;
  const AdvCfg adv = adv_cfg(opts);
  const int chunk = adv.chunk;
  const bool tracing = opts_in && opts_in->trace;

  const bool idem = bfs_idem_on(opts, pull_ok);
  const uint32_t idem_culls = (GR_IDEM_CULL_WAVE | GR_IDEM_CULL_HISTORY | GR_IDEM_CULL_LABEL) &
                              ~(uint32_t)opts.idem_culls_off;
  const int idem_log_h = opts.idem_table_log2 > 0 ? opts.idem_table_log2 : 10;
  BfsArrays a;
  GR_TRY(bfs_layout(ar, V, E, pull_ok, g->perm != nullptr, parent != nullptr, tracing, idem, &a));
  uint32_t* bm = a.bm;
  int32_t *qA = a.qA, *qB = a.qB, *qC = a.qC, *offsets = a.offsets, *rstart = a.rstart,
          *chunks = a.chunks;
  int64_t* bsums = a.bsums;
  Ctrl* ctrl = a.ctrl;
  // the fixed region keeps the last call's contents: start from zero marks
  if (a.marks)
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(a.marks), (V + 31) / 32 * 8, 0u, st));
  Ctrl* hc = ctx->host_ctrl;
  // a renumbered graph traverses into internal arrays indexed by the new
  // ids (parent values are caller ids already) and scatters them at the end
  const int32_t* perm = g->perm;
  int32_t* out_depth = depth;
  int32_t* out_parent = parent;
  if (perm && !internal_ids) {
    depth = a.depth;
    if (parent) parent = a.parent;
  }
  const int32_t src = g->to_new(source);

  int32_t* q[3] = {qA, qB, qC};
  // pull levels after the first work from the list of still-unvisited
  // vertices the previous pull level left (two lists, ping-pong)
  int32_t* ul[2] = {a.ul0, a.ul1};
  int ulc = 0;            // the list the next pull level reads
  bool list_ok = false;   // it holds every unvisited vertex with neighbours
  int64_t list_n = 0;

  GR_HIP(hipEventRecord(ctx->ev_start, st));
  GR_HIP(launch_bfs_init(depth, parent, V, bm, NW, src, qA, ctrl, st));
  int cur = 0, sp = 0, p = 0;
  GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                               &ctrl->q_count[(cur + 1) % 3], nullptr, st));
  const bool learned = opts.policy == GR_POLICY_LEARNED && ctx->policy_loaded;
  const float* mlp = static_cast<const float*>(ctx->pool[S_MLP].ptr);
  const int allowed = pull_ok ? 0xF : 0x3;
  // the selector's inputs at the current statistics slot (learned policy only)
  auto select_at = [&](int slot, int64_t n_u, int64_t m_u, int prev_pull) {
    return MlpSelect{mlp, slot, V, E, n_u, m_u, prev_pull, allowed};
  };
  MlpSelect msel = select_at(sp, V, E, 0);
  GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));

  Selector sel;
  sel.init(opts, g->V, g->E, pull_ok, /*is_sssp=*/false, ctx->policy_loaded);
  LevelFeatures lf{};
  lf.V = V;
  lf.E = E;
  int64_t n_f = hc->n_f[sp], m_f = hc->m_f[sp], max_deg = hc->max_deg[sp];
  int64_t visited_n = n_f, visited_m = m_f;
  int64_t inspected_push = 0;
  int64_t pull_in = 0;     // input vertices of the last pull level (trace)
  int64_t pull_seen = 0;   // the device's pull neighbour count before this level
  int level = 0;
  gr_run_stats rs{};
  DlPlan dl;
  GR_TRY(dl_plan(ctx, ar, opts, pull_ok, learned, tracing, &dl));

  while (n_f > 0 && (opts.max_iterations <= 0 || level < opts.max_iterations)) {
    lf.level = level;
    lf.n_f = n_f;
    lf.m_f = m_f;
    lf.max_deg_f = max_deg;
    lf.n_u = V - visited_n;
    lf.m_u = E - visited_m;
    lf.prev_pull = sel.mode_pull ? 1 : 0;
    const bool dl_fits = dl.on && n_f <= kDlMaxN && m_f <= dl.max_m;
    const int action = sel.decide(lf, learned ? hc->action : -1, learned ? hc->pred : nullptr,
                                  dl_fits);
    if (action == GR_PUSH_LB || action == GR_PUSH_TWC) list_ok = false;
    if (dl_fits && (action == GR_PUSH_LB || action == GR_PUSH_TWC)) {
      // A block of device-predicated push levels (atomic parents, no merge
      // pass); its first level is the one just decided on the host.
      int kmax = dl.len;
      if (opts.max_iterations > 0) kmax = (int)std::min<int64_t>(kmax, opts.max_iterations - level);
      const int64_t vm0 = visited_m - m_f, vn0 = visited_n - n_f;
      // the network pushing where the heuristic would pull: the block keeps
      // pushing (its device-side direction test would stop it at once)
      const double blk_do_a = sel.last_heuristic >= GR_PULL_TWC ? -1.0 : dl.do_a;
      BlockCapture capture;
      hipStream_t es = st;
      if (dl.graph) GR_TRY(block_capture_begin(ctx, &capture, &es));
      GR_HIP(launch_dl_begin(ctrl, cur, vm0, vn0, 0u, 0, 0, es));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_a, st));
      for (int i = 0; i < kmax; ++i) {
        const int qc = (cur + i) % 3;
        const DlArgs da{g->R, g->C, q[qc], q[(qc + 1) % 3], qc, i, kDlMaxN, dl.max_m, E, blk_do_a,
                        V, dl.log, ctrl};
        GR_HIP(launch_bfs_dstep(da, bm, p ^ (i & 1), depth, parent, perm, level + i + 1, dl.blocks,
                                es));
      }
      if (dl.graph) GR_TRY(block_capture_launch(ctx, &capture, (kGraphKeyBfs << 8) | kmax, st));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_b, st));
      // statistics of the frontier the block leaves (found on the device),
      // then a single read-back; with k == 0 levels run the frontier is
      // unchanged and its statistics simply move to the other slot
      sp ^= 1;
      GR_HIP(launch_frontier_stats_after_block(Queues3{{qA, qB, qC}}, cur, g->R, bsums, ctrl, sp,
                                               st));
      msel = select_at(sp, 0, 0, 0);
      msel.after_block = 1;
      // while tracing, the publication also copies the block's level log
      const PublishExtra lgx{reinterpret_cast<const uint32_t*>(dl.log),
                             reinterpret_cast<uint32_t*>(ctx->host_dlog_dev), 6 * kmax};
      GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr, nullptr, tracing ? &lgx : nullptr));
      const int k = hc->dl_levels;
      if (k > 0) {
        const int64_t* lg = ctx->host_dlog;  // the block's level log (host copy)
        float block_ms = 0.f;
        if (tracing) GR_TRY(elapsed_ms(ctx->ev_a, ctx->ev_b, &block_ms));
        // full blocks double the next one; blocks that stop early halve it
        if (k == kmax) dl.len = std::min(2 * dl.len, kDlMaxLevels);
        else if (2 * k < kmax) dl.len = std::max(dl.len / 2, kDlFirstLen);
        rs.action_count[action] += k;
        inspected_push += hc->dl_vm[k & 1] - vm0;
        visited_n = hc->dl_vn[k & 1];
        visited_m = hc->dl_vm[k & 1];
        p ^= k & 1;
        cur = (cur + k) % 3;
        level += k;
        if (tracing) {
          int64_t vn = vn0, vm = vm0;
          for (int i = 0; i < k; ++i) {
            LevelFeatures li = lf;
            li.level = level - k + i;
            li.n_f = lg[3 * i];
            li.m_f = lg[3 * i + 1];
            li.max_deg_f = lg[3 * i + 2];
            vn += li.n_f;
            vm += li.m_f;
            li.n_u = V - vn;
            li.m_u = E - vm;
            if (i > 0) li.prev_pull = 0;
            const int64_t nn = i + 1 < k ? lg[3 * (i + 1)] : (int64_t)hc->n_f[sp];
            GR_TRY(record_trace_times(opts_in, li, action, kTraceKernelDstep, nn, block_ms / k,
                                      block_ms / k, StepWork{li.n_f, li.m_f}));
          }
        }
        n_f = hc->n_f[sp];
        m_f = hc->m_f[sp];
        max_deg = hc->max_deg[sp];
        visited_n += n_f;
        visited_m += m_f;
        continue;
      }
    }
    if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_a, st));
    const int next_depth = level + 1;
    int kernel = 0;
    if (action == GR_PUSH_LB || action == GR_PUSH_TWC) {
      const int mode = action == GR_PUSH_TWC ? 0 : (n_f < opts.lb_light_threshold ? 1 : 2);
      if (mode == 2)
        GR_HIP(launch_frontier_offsets(q[cur], n_f, g->R, bsums, &ctrl->m_f[sp], offsets, rstart,
                                       chunks, chunk, st));
      // canonical parents by an atomic minimum in the push (about one atomic
      // per frontier edge) or by the fix-up scan of the new vertices, which
      // reads each sorted list up to its first frontier neighbour: about E / m_f
      // entries when the frontier holds m_f of the E edge ends, for at most
      // min(m_f, unvisited) new vertices.  A small frontier of hubs makes the
      // scans long (R-MAT 22 BFS: 0.53-0.56 ms with this rule against
      // 0.58-0.60 ms with a fixed 4 M-edge bound and 0.61-0.63 ms with 1 M).
      const double new_max = (double)std::min<int64_t>(m_f, V - visited_n);
      const bool atomic_cheaper = (double)m_f * (double)m_f <= 2.0 * new_max * (double)E;
      const bool atomic_parent =
          !idem && parent && (!pull_ok || m_f <= kAtomicParentMaxEdges || atomic_cheaper);
      if (idem) {
        // idempotent advance into the candidate list, then the exact filter
        kernel = kTraceKernelIdem + mode;
        GR_HIP(launch_fill_u32(&ctrl->cand_count, 1, 0u, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
        GR_HIP(launch_bfs_push_idem(mode, q[cur], offsets, rstart, chunks, n_f, m_f, g->R, g->C, bm,
                                    p, depth, next_depth, idem_culls, idem_log_h, a.cand,
                                    &ctrl->cand_count, V, adv, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
        GR_HIP(launch_bfs_idem_filter(a.cand, &ctrl->cand_count, V, V, bm, p, depth, next_depth,
                                      q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3], st));
      } else if (opts.bfs_filter != GR_BFS_FILTER_ATOMIC && m_f >= V / kMarksFilterDivisor) {
        // byte marks; parents by the fix-up scan, or by atomic minima in the
        // push (no returning atomic either way)
        uint8_t* marks;
        GR_TRY(marks_buffer(ctx, ar, V, &marks, st));
        kernel = mode == 2 ? 3 : mode;
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
        GR_HIP(launch_bfs_push_marks(mode, q[cur], offsets, rstart, chunks, n_f, m_f, g->R, g->C,
                                     bm, p, marks, atomic_parent ? parent : nullptr, perm, adv,
                                     st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
        GR_HIP(launch_bfs_mark_compact(marks, V, bm, p, depth, next_depth, q[(cur + 1) % 3],
                                       &ctrl->q_count[(cur + 1) % 3], st));
      } else {
        kernel = mode;
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
        GR_HIP(launch_bfs_push(mode, atomic_parent, q[cur], offsets, rstart, chunks, n_f, m_f,
                               g->R, g->C, bm, p, depth, parent, perm, next_depth, q[(cur + 1) % 3],
                               &ctrl->q_count[(cur + 1) % 3], adv, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      }
      if (parent && !atomic_parent)
        GR_HIP(launch_bfs_parent_fixup(q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3],
                                       std::min<int64_t>(V - visited_n, m_f), g->R, g->C, bm, p,
                                       parent, perm, st));
      inspected_push += m_f;
    } else {
      kernel = action == GR_PULL_LB ? 5 : 4;
      pull_in = lf.n_u;
      // every pull lists the vertices it leaves unvisited, and the next pull
      // level reads that list instead of the bitmap once it is short
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
      if (list_ok && list_n <= V / kPullListDivisor) {
        kernel = kTraceKernelPullList;
        pull_in = list_n;
      }
      if (kernel == kTraceKernelPullList)
        GR_HIP(launch_bfs_pull_list(ul[ulc], &ctrl->ul_count[ulc], list_n, g->R, g->C, bm, p,
                                    depth, parent, perm, next_depth, q[(cur + 1) % 3],
                                    &ctrl->q_count[(cur + 1) % 3], &ctrl->inspected, ul[ulc ^ 1],
                                    &ctrl->ul_count[ulc ^ 1], st));
      else
        GR_HIP(launch_bfs_pull(action == GR_PULL_LB, V, g->R, g->C, bm, p, depth, parent, perm,
                               next_depth, q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3],
                               &ctrl->inspected, ul[ulc ^ 1], &ctrl->ul_count[ulc ^ 1], st));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      ulc ^= 1;
      list_ok = true;
    }
    GR_HIP(launch_bitmap_merge(bm, p, NW, st));
    if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_b, st));
    rs.action_count[action]++;
    p ^= 1;
    cur = (cur + 1) % 3;
    sp ^= 1;
    ++level;
    // (the list the next pull level appends to starts empty)
    GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                 &ctrl->q_count[(cur + 1) % 3], &ctrl->ul_count[ulc ^ 1], st));
    msel = select_at(sp, V - visited_n, E - visited_m, sel.mode_pull ? 1 : 0);
    GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));
    list_n = hc->ul_count[ulc];
    if (tracing) {
      const bool pulled = kernel >= 4 && kernel <= kTraceKernelPullList;
      const bool idem_step = kernel >= kTraceKernelIdem;
      const StepWork w{pulled ? pull_in : n_f,
                       pulled ? (int64_t)hc->inspected - pull_seen : m_f,
                       idem_step ? (int64_t)hc->cand_count : -1};
      GR_TRY(record_trace(ctx, opts_in, lf, action, kernel, hc->n_f[sp], w));
    }
    pull_seen = hc->inspected;
    n_f = hc->n_f[sp];
    m_f = hc->m_f[sp];
    max_deg = hc->max_deg[sp];
    visited_n += n_f;
    visited_m += m_f;
  }
  if (perm && !internal_ids)
    GR_HIP(launch_permute_out(g->inv, V, depth, parent, out_depth, out_parent, st));
  GR_HIP(hipEventRecord(ctx->ev_stop, st));
  GR_HIP(hipEventSynchronize(ctx->ev_stop));
  if (stats) {
    float ms = 0.f;
    GR_TRY(elapsed_ms(ctx->ev_start, ctx->ev_stop, &ms));
    rs.iterations = level;
    // when stopped early the last frontier is reached but not expanded
    rs.teps_edges = visited_m;
    rs.inspected_edges = inspected_push + hc->inspected;
    rs.device_ms = ms;
    *stats = rs;
  }
  return GR_OK;
}

}  // namespace

extern "C" gr_status gr_bfs(gr_ctx* ctx, const gr_graph* g, int32_t source, int32_t* depth,
                            int32_t* parent, gr_opts* opts_in, void* stream, gr_run_stats* stats) {
  GR_TRY(bfs_check("gr_bfs", ctx, g, source, depth));
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  DeviceGuard dg(ctx->device);
  Arena ar;
  ar.ctx = ctx;
  return bfs_run(ctx, g, source, depth, parent, opts_in, opts, static_cast<hipStream_t>(stream),
                 stats, ar);
}

extern "C" gr_status gr_bfs_static(gr_ctx* ctx, const gr_graph* g, int32_t source, int32_t* depth,
                                   int32_t* parent, gr_opts* opts_in, void* stream,
                                   gr_run_stats* stats) {
  GR_TRY(bfs_check("gr_bfs_static", ctx, g, source, depth));
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  if (!ctx->static_ws) return fail(GR_EHIP, "gr_bfs_static: the context has no static workspace");
  // lay the working arrays out without touching the device, and refuse
  // graphs whose arrays do not fit before any work is enqueued
  Arena m;
  m.measure = true;
  BfsArrays unused;
  const bool tracing = opts_in && opts_in->trace;
  GR_TRY(bfs_layout(m, g->V, g->E, (g->flags & GR_SYMMETRIC) != 0, g->perm != nullptr,
                    parent != nullptr, tracing, bfs_idem_on(opts, (g->flags & GR_SYMMETRIC) != 0),
                    &unused));
  if (m.used > (size_t)GR_STATIC_WORKSPACE_BYTES)
    return fail(GR_ERANGE, "gr_bfs_static: this graph needs " + std::to_string(m.used) +
                               " bytes of working arrays, the static workspace holds " +
                               std::to_string((size_t)GR_STATIC_WORKSPACE_BYTES));
  DeviceGuard dg(ctx->device);
  Arena ar;
  ar.ctx = ctx;
  ar.base = static_cast<char*>(ctx->static_ws);
  ar.cap = GR_STATIC_WORKSPACE_BYTES;
  return bfs_run(ctx, g, source, depth, parent, opts_in, opts, static_cast<hipStream_t>(stream),
                 stats, ar);
}

// ============================================================================
// SSSP enactor (Sec. 6.2, Alg. 1)
// ============================================================================

extern "C" gr_status gr_sssp(gr_ctx* ctx, const gr_graph* g, const int32_t* sources,
                             int32_t n_sources, uint32_t* dist, int32_t* pred, gr_opts* opts_in,
                             void* stream, gr_run_stats* stats) {
  if (!ctx || !g) return fail(GR_EINVAL, "gr_sssp: ctx or graph is NULL");
  if (g->ctx != ctx) return fail(GR_EINVAL, "gr_sssp: graph belongs to another context");
  if (!dist) return fail(GR_EINVAL, "gr_sssp: dist is NULL");
  if (!sources || n_sources < 1) return fail(GR_EINVAL, "gr_sssp: need at least one source");
  if (!g->W) return fail(GR_EINVAL, "gr_sssp: graph has no weights");
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || (int64_t)sources[i] >= g->V)
      return fail(GR_EINVAL, "gr_sssp: source " + std::to_string(sources[i]) + " out of range");
  if ((uint64_t)g->max_weight * (uint64_t)(g->V - 1) >= 0xffffffffull)
    return fail(GR_ERANGE, "gr_sssp: max_weight * (V - 1) >= 2^32 - 1, distances may not fit uint32");
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t V = g->V, E = g->E;
  const int G = stats_grid();
  const AdvCfg adv = adv_cfg(opts);
  const int chunk = adv.chunk;

  std::vector<int32_t> uniq(sources, sources + n_sources);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  const int32_t n_src = (int32_t)uniq.size();

  int32_t *qA, *qB, *qC, *offsets, *rstart, *chunks, *tags, *src_dev;
  unsigned long long* keys;
  int64_t* bsums;
  Ctrl* ctrl;
  GR_TRY(pool_typed(ctx, S_Q_A, V, &qA));
  GR_TRY(pool_typed(ctx, S_Q_B, V, &qB));
  GR_TRY(pool_typed(ctx, S_Q_C, V, &qC));
  GR_TRY(pool_typed(ctx, S_OFFSETS, V + 1, &offsets));
  GR_TRY(pool_typed(ctx, S_RSTART, V, &rstart));
  GR_TRY(pool_typed(ctx, S_CHUNKS, E / 512 + 2, &chunks));
  GR_TRY(pool_typed(ctx, S_BLOCK_SUMS, G + 1, &bsums));
  GR_TRY(pool_typed(ctx, S_CTRL, 1, &ctrl));
  GR_TRY(pool_typed(ctx, S_KEYS, V, &keys));
  GR_TRY(pool_typed(ctx, S_TAGS, V, &tags));
  uint8_t* mirror_p;
  GR_TRY(pool_typed(ctx, S_MIRROR, V, &mirror_p));
  const DistMirror mirror{mirror_p, mirror_shift_for(g->max_weight)};
  uint32_t* relaxed = nullptr;
  if (!(opts.sssp_opt_off & GR_SSSP_OPT_CULL)) GR_TRY(pool_typed(ctx, S_RELAXED, V, &relaxed));
  // src_dev: the sources in traversal ids, then in caller ids
  GR_TRY(pool_typed(ctx, S_TMP0, 2 * (size_t)n_src, &src_dev));
  std::vector<int32_t> src_both(2 * (size_t)n_src);
  for (int32_t i = 0; i < n_src; ++i) {
    src_both[i] = g->to_new(uniq[i]);
    src_both[n_src + i] = uniq[i];
  }
  const int32_t* perm = g->perm;
  // two-level priority queue (near / far piles), when sssp_delta > 0
  const bool use_pq = opts.sssp_delta > 0;
  PqState pq{};
  pq.perm = perm;
  if (use_pq) {
    pq.T = (uint32_t)opts.sssp_delta;
    pq.delta = (uint32_t)opts.sssp_delta;
    pq.V = V;
    GR_TRY(pool_typed(ctx, S_FAR, 3 * V, &pq.far_base));
    GR_TRY(pool_typed(ctx, S_FAR_TAGS, V, &pq.far_tag));
  }
  // distance bins of the marks compaction
  SsspBins bins{nullptr, 0u};
  if (!use_pq && !(opts.sssp_opt_off & GR_SSSP_OPT_BINS)) {
    GR_TRY(pool_typed(ctx, S_SSSP_BINS, kSsspBinWords, &bins.state));
    bins.shift = bin_shift_for(g->max_weight);
  }
  Ctrl* hc = ctx->host_ctrl;
  int32_t* q[3] = {qA, qB, qC};

  GR_HIP(hipMemcpyAsync(src_dev, src_both.data(), sizeof(int32_t) * 2 * n_src,
                        hipMemcpyHostToDevice, st));
  GR_HIP(hipMemcpyAsync(qA, src_both.data(), sizeof(int32_t) * n_src, hipMemcpyHostToDevice, st));
  GR_HIP(hipStreamSynchronize(st));  // the host vector must outlive the copies
  GR_HIP(hipEventRecord(ctx->ev_start, st));
  GR_HIP(launch_sssp_init(keys, tags, use_pq ? pq.far_tag : nullptr, mirror, relaxed, bins.state,
                          V, ctrl, st));
  GR_HIP(launch_sssp_seed(src_dev, n_src, keys, tags, ctrl, st));
  int cur = 0, sp = 0;
  GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                               &ctrl->q_count[(cur + 1) % 3], nullptr, st));
  const bool learned = opts.policy == GR_POLICY_LEARNED && ctx->policy_loaded;
  const float* mlp = static_cast<const float*>(ctx->pool[S_MLP].ptr);
  MlpSelect msel{mlp, sp, V, E, 0, 0, 0, 0x3};
  GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));

  Selector sel;
  sel.init(opts, V, E, /*pull_ok=*/false, /*is_sssp=*/true, ctx->policy_loaded);
  LevelFeatures lf{};
  lf.V = V;
  lf.E = E;
  int64_t n_f = hc->n_f[sp], m_f = hc->m_f[sp], max_deg = hc->max_deg[sp];
  int64_t far_n = 0;
  int it = 0;
  int64_t inspected = 0;
  int64_t expanded = 0;  // sum of the frontier sizes so far
  gr_run_stats rs{};
  const bool tracing = opts_in && opts_in->trace;
  DlPlan dl;
  Arena ar;
  ar.ctx = ctx;
  GR_TRY(dl_plan(ctx, ar, opts, /*pull_ok=*/false, learned, tracing, &dl));
  // after a step that produced the frontier in q[cur]: statistics, selector, read-back
  // with load-balanced advance likely (average degree), the degree scan of
  // each new frontier is queued ahead of the read-back (offsets_ready)
  const bool lb_likely = (double)E / (double)V >= (double)opts.lb_min_avg_degree;
  bool offsets_ready = false;
  auto next_frontier = [&]() -> gr_status {
    GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                 &ctrl->q_count[(cur + 1) % 3], nullptr, st));
    msel.sp = sp;
    const OffsetsJob pre{q[cur], &ctrl->q_count[cur], g->R, bsums, &ctrl->m_f[sp], offsets,
                         rstart, chunks, chunk};
    GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr, lb_likely ? &pre : nullptr));
    offsets_ready = lb_likely;
    if (use_pq) far_n = hc->far_count[pq.fc];
    return GR_OK;
  };
  while ((n_f > 0 || far_n > 0) && (opts.max_iterations <= 0 || it < opts.max_iterations)) {
    lf.level = it;
    lf.n_f = n_f;
    lf.m_f = m_f;
    lf.max_deg_f = max_deg;
    lf.n_u = 0;
    lf.m_u = 0;
    lf.prev_pull = 0;
    const bool dl_fits = dl.on && n_f <= kDlMaxN && m_f <= dl.max_m;
    const int action = sel.decide(lf, learned ? hc->action : -1, learned ? hc->pred : nullptr);
    if (dl_fits) {
      // A block of device-predicated relaxation rounds (Alg. 1 iterations;
      // with the priority queue also its refill steps).
      offsets_ready = false;  // the block leaves a frontier the scan has not seen
      int kmax = dl.len;
      if (opts.max_iterations > 0) kmax = std::min(kmax, opts.max_iterations - it);
      BlockCapture capture;
      hipStream_t es = st;
      if (dl.graph) GR_TRY(block_capture_begin(ctx, &capture, &es));
      GR_HIP(launch_dl_begin(ctrl, cur, 0, 0, pq.T, pq.epoch, pq.fc, es));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_a, st));
      for (int i = 0; i < kmax; ++i) {
        const int qc = (cur + i) % 3;
        const DlArgs da{g->R, g->C, q[qc], q[(qc + 1) % 3], qc, i, kDlMaxN, dl.max_m, E, -1.0,
                        V, dl.log, ctrl};
        if (use_pq) GR_HIP(launch_sssp_pq_dstep(da, g->W, keys, tags, it + i + 1, pq, dl.blocks, es));
        else GR_HIP(launch_sssp_dstep(da, g->W, keys, tags, perm, it + i + 1, dl.blocks, es));
      }
      if (dl.graph)
        GR_TRY(block_capture_launch(ctx, &capture,
                                    ((use_pq ? kGraphKeySsspPq : kGraphKeySssp) << 8) | kmax, st));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_b, st));
      // statistics of the frontier the block leaves, then a single read-back
      // (with k == 0 levels run the statistics just move to the other slot)
      sp ^= 1;
      GR_HIP(launch_frontier_stats_after_block(Queues3{{qA, qB, qC}}, cur, g->R, bsums, ctrl, sp,
                                               st));
      msel.sp = sp;
      // while tracing, the publication also copies the block's level log
      const PublishExtra lgx{reinterpret_cast<const uint32_t*>(dl.log),
                             reinterpret_cast<uint32_t*>(ctx->host_dlog_dev), 6 * kmax};
      GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr, nullptr, tracing ? &lgx : nullptr));
      const int k = hc->dl_levels;
      if (use_pq) {
        pq.T = hc->pq_T[k & 1];
        pq.epoch = hc->pq_epoch[k & 1];
        pq.fc = hc->pq_fc[k & 1];
        far_n = hc->far_count[pq.fc];
      }
      if (k > 0) {
        const int64_t* lg = ctx->host_dlog;  // the block's level log (host copy)
        float block_ms = 0.f;
        if (tracing) GR_TRY(elapsed_ms(ctx->ev_a, ctx->ev_b, &block_ms));
        // full blocks double the next one; blocks that stop early halve it
        if (k == kmax) dl.len = std::min(2 * dl.len, kDlMaxLevels);
        else if (2 * k < kmax) dl.len = std::max(dl.len / 2, kDlFirstLen);
        rs.action_count[action] += k;
        inspected += hc->dl_vm[k & 1];
        expanded += hc->dl_vn[k & 1];
        cur = (cur + k) % 3;
        it += k;
        if (tracing) {
          for (int i = 0; i < k; ++i) {
            LevelFeatures li = lf;
            li.level = it - k + i;
            li.n_f = lg[3 * i];
            li.m_f = lg[3 * i + 1];
            li.max_deg_f = lg[3 * i + 2];
            const int64_t nn = i + 1 < k ? lg[3 * (i + 1)] : (int64_t)hc->n_f[sp];
            GR_TRY(record_trace_times(opts_in, li, action, kTraceKernelDstep, nn, block_ms / k,
                                      block_ms / k, StepWork{li.n_f, li.m_f}));
          }
        }
        n_f = hc->n_f[sp];
        m_f = hc->m_f[sp];
        max_deg = hc->max_deg[sp];
        continue;
      }
    }
    if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_a, st));
    int kernel = kTraceKernelRefill;
    const int64_t refill_in = far_n;
    if (n_f == 0) {
      // priority queue: the near frontier ran dry, raise the threshold and
      // split the far pile
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
      GR_HIP(launch_sssp_pq_refill(keys, pq, ctrl, far_n, q[(cur + 1) % 3],
                                   &ctrl->q_count[(cur + 1) % 3], st));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      const uint64_t t1 = (uint64_t)pq.T + pq.delta;
      pq.T = t1 >= 0xffffffffull ? 0xffffffffu : (uint32_t)t1;
      pq.epoch += 1;
      pq.fc = (pq.fc + 1) % 3;
    } else {
      const int mode = action == GR_PUSH_TWC ? 0 : (n_f < opts.lb_light_threshold ? 1 : 2);
      kernel = mode;
      if (mode == 2 && !offsets_ready)
        GR_HIP(launch_frontier_offsets(q[cur], n_f, g->R, bsums, &ctrl->m_f[sp], offsets, rstart,
                                       chunks, chunk, st));
      if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
      if (m_f >= V / kSsspMarksDivisor) {
        // many frontier edges: relax with no returning atomic, then list the
        // vertices whose distance dropped (byte marks); with the priority
        // queue the list is split into the next frontier and the far pile
        uint8_t* marks;
        GR_TRY(marks_buffer(ctx, ar, V, &marks, st));
        kernel += kTraceMarksOffset;
        const bool screen = expanded + n_f + far_n >= V / kSsspMirrorDivisor;
        GR_HIP(launch_sssp_relax_marks(mode, q[cur], offsets, rstart, chunks, n_f, m_f, g->R, g->C,
                                       g->W, keys, perm, marks, mirror, relaxed, screen, adv,
                                       st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
        if (use_pq)
          GR_HIP(launch_sssp_pq_mark_compact(marks, V, keys, mirror, relaxed, pq, ctrl,
                                             q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3], st));
        else if (bins.state)
          GR_HIP(launch_sssp_bin_compact(marks, V, keys, mirror, relaxed, bins, q[(cur + 1) % 3],
                                         &ctrl->q_count[(cur + 1) % 3], st));
        else
          GR_HIP(launch_sssp_mark_compact(marks, V, keys, mirror, relaxed, q[(cur + 1) % 3],
                                          &ctrl->q_count[(cur + 1) % 3], st));
      } else if (use_pq) {
        GR_HIP(launch_sssp_pq_relax(mode, q[cur], offsets, rstart, chunks, n_f, m_f, g->R, g->C,
                                    g->W, keys, tags, it + 1, pq, ctrl, q[(cur + 1) % 3],
                                    &ctrl->q_count[(cur + 1) % 3], adv, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      } else {
        GR_HIP(launch_sssp_relax(mode, q[cur], offsets, rstart, chunks, n_f, m_f, g->R, g->C, g->W,
                                 keys, tags, perm, it + 1, q[(cur + 1) % 3],
                                 &ctrl->q_count[(cur + 1) % 3], adv, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      }
      inspected += m_f;
      expanded += n_f;
      rs.action_count[action]++;
    }
    if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_b, st));
    cur = (cur + 1) % 3;
    sp ^= 1;
    ++it;
    GR_TRY(next_frontier());
    if (tracing)
      GR_TRY(record_trace(ctx, opts_in, lf, action, kernel, hc->n_f[sp],
                          kernel == kTraceKernelRefill ? StepWork{refill_in, 0} : StepWork{n_f, m_f}));
    n_f = hc->n_f[sp];
    m_f = hc->m_f[sp];
    max_deg = hc->max_deg[sp];
  }
  int64_t* reached = &ctrl->reached_edges;
  GR_HIP(launch_sssp_finalize(keys, perm ? g->R_orig : g->R, V, dist, pred, perm ? g->inv : nullptr,
                              src_dev + n_src, n_src, reached, st));
  GR_HIP(hipEventRecord(ctx->ev_stop, st));
  GR_TRY(read_ctrl(ctx, ctrl, st));
  if (stats) {
    float ms = 0.f;
    GR_TRY(elapsed_ms(ctx->ev_start, ctx->ev_stop, &ms));
    rs.iterations = it;
    rs.teps_edges = hc->reached_edges;
    rs.inspected_edges = inspected;
    rs.device_ms = ms;
    *stats = rs;
  }
  return GR_OK;
}

// ============================================================================
// multi-source BFS
// ============================================================================

extern "C" gr_status gr_bfs_multi(gr_ctx* ctx, const gr_graph* g, const int32_t* sources,
                                  int32_t k, int32_t* depth, int32_t* parent, gr_opts* opts_in,
                                  void* stream, gr_run_stats* stats) {
  if (!ctx || !g) return fail(GR_EINVAL, "gr_bfs_multi: ctx or graph is NULL");
  if (g->ctx != ctx) return fail(GR_EINVAL, "gr_bfs_multi: graph belongs to another context");
  if (!depth) return fail(GR_EINVAL, "gr_bfs_multi: depth is NULL");
  if (!sources || k < 1) return fail(GR_EINVAL, "gr_bfs_multi: need at least one source");
  for (int32_t i = 0; i < k; ++i)
    if (sources[i] < 0 || (int64_t)sources[i] >= g->V)
      return fail(GR_EINVAL, "gr_bfs_multi: source " + std::to_string(sources[i]) + " out of range");
  if (!(g->flags & GR_SYMMETRIC))
    return fail(GR_EUNSUPPORTED, "gr_bfs_multi needs a symmetric graph (parents are pulled over in-edges)");
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t V = g->V, E = g->E;
  const int G = stats_grid();
  const AdvCfg adv = adv_cfg(opts);
  const int chunk = adv.chunk;
  const bool use_lb = (double)E / (double)V >= (double)opts.lb_min_avg_degree;
  using u64 = unsigned long long;

  u64 *visit, *front[2], *next;
  int32_t *qA, *qB, *qC, *offsets, *rstart, *chunks, *src_dev;
  int64_t* bsums;
  Ctrl* ctrl;
  GR_TRY(pool_typed(ctx, S_MASK_A, V, &visit));
  GR_TRY(pool_typed(ctx, S_MASK_B, V, &front[0]));
  GR_TRY(pool_typed(ctx, S_MASK_C, V, &front[1]));
  GR_TRY(pool_typed(ctx, S_KEYS, V, &next));
  GR_TRY(pool_typed(ctx, S_Q_A, V, &qA));
  GR_TRY(pool_typed(ctx, S_Q_B, V, &qB));
  GR_TRY(pool_typed(ctx, S_Q_C, V, &qC));
  GR_TRY(pool_typed(ctx, S_OFFSETS, V + 1, &offsets));
  GR_TRY(pool_typed(ctx, S_RSTART, V, &rstart));
  GR_TRY(pool_typed(ctx, S_CHUNKS, E / 512 + 2, &chunks));
  GR_TRY(pool_typed(ctx, S_BLOCK_SUMS, G + 1, &bsums));
  GR_TRY(pool_typed(ctx, S_CTRL, 1, &ctrl));
  GR_TRY(pool_typed(ctx, S_TMP0, 128, &src_dev));  // traversal ids, then caller ids
  Ctrl* hc = ctx->host_ctrl;
  int32_t* q[3] = {qA, qB, qC};

  GR_HIP(hipEventRecord(ctx->ev_start, st));
  GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(depth), (int64_t)k * V, 0xffffffffu, st));
  if (parent)
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(parent), (int64_t)k * V, 0xffffffffu, st));
  GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->reached_edges), 2, 0u, st));
  gr_run_stats rs{};
  int64_t inspected = 0;
  int max_levels = 0;
  const bool learned = opts.policy == GR_POLICY_LEARNED && ctx->policy_loaded;
  const float* mlp = static_cast<const float*>(ctx->pool[S_MLP].ptr) + ctx->mlp_multi_offset;
  const bool tracing = opts_in && opts_in->trace;
  uint64_t rng = opts.policy_seed ^ 0x9e3779b97f4a7c15ull;
  // small push levels run in blocks of device-predicated levels (as gr_bfs):
  // not while tracing (a record per level) or under the random policy
  const bool dl_on = opts.device_max_edges >= 0 && !tracing && opts.policy != GR_POLICY_RANDOM;
  const int64_t dl_max_m = opts.device_max_edges > 0 ? opts.device_max_edges : kDlDefaultMaxEdges;
  const double dl_do_a = opts.policy == GR_POLICY_FIXED ? -1.0 : (double)opts.do_a;
  const int dl_blocks = ctx->cu_count > 0 ? ctx->cu_count : 256;
  int dl_len = kDlFirstLen;
  for (int32_t p0 = 0; p0 < k; p0 += 64) {
    const int32_t kk = std::min<int32_t>(64, k - p0);
    const u64 full = kk == 64 ? ~0ull : ((1ull << kk) - 1ull);
    int32_t* dpass = depth + (int64_t)p0 * V;
    int32_t* ppass = parent ? parent + (int64_t)p0 * V : nullptr;
    // srcs: this pass's sources in traversal ids [kk], then in caller ids [kk]
    std::vector<int32_t> srcs(2 * (size_t)kk);
    for (int32_t i = 0; i < kk; ++i) {
      srcs[i] = g->to_new(sources[p0 + i]);
      srcs[kk + i] = sources[p0 + i];
    }
    std::vector<int32_t> uniq(srcs.begin(), srcs.begin() + kk);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    for (u64* m : {visit, front[0], front[1], next})
      GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(m), 2 * V, 0u, st));
    GR_HIP(hipMemcpyAsync(src_dev, srcs.data(), sizeof(int32_t) * 2 * kk, hipMemcpyHostToDevice, st));
    GR_HIP(hipMemcpyAsync(qA, uniq.data(), sizeof(int32_t) * uniq.size(), hipMemcpyHostToDevice, st));
    GR_HIP(launch_fill_u32(&ctrl->q_count[0], 1, (uint32_t)uniq.size(), st));
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->m_f[0]), 8, 0u, st));  // m_f, max_deg
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->ms_pairs), 4, 0u, st));
    GR_HIP(launch_ms_seed(src_dev, src_dev + kk, kk, visit, front[0], dpass, V, g->R, ctrl, st));
    int cur = 0, fc = 0, sp = 0, level = 0;
    bool prev_pull = false;
    // the network's inputs for the frontier measured at slot `slot`
    auto select_at = [&](int slot) {
      MlpSelect m{mlp, slot, V, E, 0, 0, prev_pull ? 1 : 0, 0xF};
      m.ms_k = kk;
      return m;
    };
    GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                 &ctrl->q_count[(cur + 1) % 3], nullptr, st));
    MlpSelect msel = select_at(sp);
    // (the read-back also keeps the host source vectors alive for the copies)
    GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));
    int64_t n_a = hc->n_f[sp], m_a = hc->m_f[sp];
    while (n_a > 0 && (opts.max_iterations <= 0 || level < opts.max_iterations)) {
      // heuristic: pull (every vertex with unreached source bits ORs its
      // neighbours' frontier masks) once the active vertices carry more than
      // E * do_a edges; fixed / random / learned policies as for gr_bfs (both
      // pull actions map to the one pull kernel)
      const int h = (double)m_a > (double)E * (double)opts.do_a ? GR_PULL_TWC
                                                                : (use_lb ? GR_PUSH_LB : GR_PUSH_TWC);
      int action = h;
      if (opts.policy == GR_POLICY_FIXED) {
        action = opts.fixed_action;
      } else if (opts.policy == GR_POLICY_RANDOM) {
        action = (int)(Selector::next(rng) % 4);
      } else if (learned) {
        const int c = hc->action;
        if (c >= 0 && c < 4 && c != h && hc->pred[c] + opts.learned_margin < hc->pred[h]) action = c;
        // as in gr_bfs: a push level that fits a device block stays a push
        // (the network was trained on levels with one round trip each)
        if (dl_on && n_a <= kDlMaxN && m_a <= dl_max_m && h < GR_PULL_TWC && action >= GR_PULL_TWC)
          action = h;
      }
      LevelFeatures lf{};
      lf.level = level;
      lf.V = V;
      lf.E = E;
      lf.n_f = n_a;
      lf.m_f = m_a;
      lf.n_u = V - hc->ms_pairs / kk;
      lf.m_u = E - hc->ms_pair_edges / kk;
      lf.max_deg_f = hc->max_deg[sp];
      lf.prev_pull = prev_pull ? 1 : 0;
      lf.ms_k = kk;
      const bool pull = action >= GR_PULL_TWC;
      if (dl_on && !pull && n_a <= kDlMaxN && m_a <= dl_max_m) {
        // a block of device-predicated push levels, one read-back per block;
        // its first level is the one just decided, the others follow the
        // heuristic's push test on the device
        int kmax = dl_len;
        if (opts.max_iterations > 0) kmax = std::min(kmax, opts.max_iterations - level);
        GR_HIP(launch_dl_begin(ctrl, cur, 0, 0, 0u, 0, 0, st));
        for (int i = 0; i < kmax; ++i) {
          const int qc = (cur + i) % 3;
          const int fi = fc ^ (i & 1);
          DlArgs da{g->R, g->C, q[qc], q[(qc + 1) % 3], qc, i, kDlMaxN, dl_max_m, E, dl_do_a, V,
                    nullptr, ctrl};
          da.edges_vs_all = 1;
          const MsLevel ml{g->R, g->C, front[fi], front[fi ^ 1], visit, next, dpass, ppass,
                           g->perm, V, level + i + 1};
          GR_HIP(launch_ms_dlevel(da, ml, dl_blocks, std::min<int64_t>(V, dl_max_m), st));
        }
        sp ^= 1;
        GR_HIP(launch_frontier_stats_after_block(Queues3{{qA, qB, qC}}, cur, g->R, bsums, ctrl, sp,
                                                 st));
        prev_pull = false;
        msel = select_at(sp);
        GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));
        const int kd = hc->dl_levels;
        if (kd == kmax) dl_len = std::min(2 * dl_len, kDlMaxLevels);
        else if (2 * kd < kmax) dl_len = std::max(dl_len / 2, kDlFirstLen);
        rs.action_count[action] += kd;
        inspected += hc->dl_vm[kd & 1];
        cur = (cur + kd) % 3;
        fc ^= kd & 1;
        level += kd;
        n_a = hc->n_f[sp];
        m_a = hc->m_f[sp];
        if (kd > 0) continue;
        // no level ran: the same frontier continues on the host path
        lf.max_deg_f = hc->max_deg[sp];
      }
      int kernel = 4;
      if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_a, st));
      if (pull) {
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
        GR_HIP(launch_ms_pull(V, g->R, g->C, front[fc], visit, full, next, q[(cur + 1) % 3],
                              &ctrl->q_count[(cur + 1) % 3], ppass, g->perm, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      } else {
        const int mode = action == GR_PUSH_TWC ? 0 : (n_a < opts.lb_light_threshold ? 1 : 2);
        kernel = mode;
        if (mode == 2)
          GR_HIP(launch_frontier_offsets(q[cur], n_a, g->R, bsums, &ctrl->m_f[sp], offsets, rstart,
                                         chunks, chunk, st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k0, st));
        GR_HIP(launch_ms_push(mode, q[cur], offsets, rstart, chunks, n_a, m_a, g->R, g->C,
                              front[fc], visit, next, q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3], adv,
                              st));
        if (tracing) GR_HIP(hipEventRecord(ctx->ev_k1, st));
      }
      rs.action_count[action]++;
      inspected += pull ? E : m_a;
      // a pull level has written its parents already
      GR_HIP(launch_ms_finalize(q[(cur + 1) % 3], &ctrl->q_count[(cur + 1) % 3], pull ? V : std::min(V, m_a),
                                g->R, g->C, front[fc], front[fc ^ 1], visit, next, dpass,
                                pull ? nullptr : ppass, g->perm, V, level + 1, ctrl, st));
      GR_HIP(launch_ms_clear(q[cur], &ctrl->q_count[cur], n_a, front[fc], st));
      if (tracing && !opts.trace_steps_off) GR_HIP(hipEventRecord(ctx->ev_b, st));
      prev_pull = pull;
      fc ^= 1;
      cur = (cur + 1) % 3;
      sp ^= 1;
      ++level;
      GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                   &ctrl->q_count[(cur + 1) % 3], nullptr, st));
      msel = select_at(sp);
      GR_TRY(read_ctrl(ctx, ctrl, st, learned ? &msel : nullptr));
      if (tracing)
        GR_TRY(record_trace(ctx, opts_in, lf, action, kernel, hc->n_f[sp],
                            StepWork{pull ? V : n_a, pull ? E : m_a}));
      n_a = hc->n_f[sp];
      m_a = hc->m_f[sp];
    }
    max_levels = std::max(max_levels, level);
    GR_HIP(launch_ms_teps(visit, g->R, V, &ctrl->reached_edges, st));
  }
  GR_HIP(hipEventRecord(ctx->ev_stop, st));
  GR_TRY(read_ctrl(ctx, ctrl, st));
  if (stats) {
    float ms = 0.f;
    GR_TRY(elapsed_ms(ctx->ev_start, ctx->ev_stop, &ms));
    rs.iterations = max_levels;
    rs.teps_edges = hc->reached_edges;
    rs.inspected_edges = inspected;
    rs.device_ms = ms;
    *stats = rs;
  }
  return GR_OK;
}

// ============================================================================
// batched shortest paths (Sec. 8 task parallelism applied to Alg. 1)
// ============================================================================

extern "C" gr_status gr_sssp_multi(gr_ctx* ctx, const gr_graph* g, const int32_t* sources,
                                   int32_t k, uint32_t* dist, int32_t* pred, gr_opts* opts_in,
                                   void* stream, gr_run_stats* stats) {
  if (!ctx || !g) return fail(GR_EINVAL, "gr_sssp_multi: ctx or graph is NULL");
  if (g->ctx != ctx) return fail(GR_EINVAL, "gr_sssp_multi: graph belongs to another context");
  if (!dist) return fail(GR_EINVAL, "gr_sssp_multi: dist is NULL");
  if (!sources || k < 1) return fail(GR_EINVAL, "gr_sssp_multi: need at least one source");
  if (!g->W) return fail(GR_EINVAL, "gr_sssp_multi: graph has no weights");
  for (int32_t i = 0; i < k; ++i)
    if (sources[i] < 0 || (int64_t)sources[i] >= g->V)
      return fail(GR_EINVAL, "gr_sssp_multi: source " + std::to_string(sources[i]) + " out of range");
  if ((uint64_t)g->max_weight * (uint64_t)(g->V - 1) >= 0xffffffffull)
    return fail(GR_ERANGE, "gr_sssp_multi: max_weight * (V - 1) >= 2^32 - 1, distances may not fit uint32");
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t V = g->V, E = g->E;
  if (opts.sssp_multi_sweep == 1) {
    // one source per sweep: row s is gr_sssp from sources[s]
    gr_opts o1 = opts;
    o1.trace = nullptr;
    o1.trace_capacity = 0;
    gr_run_stats agg{}, s1{};
    for (int32_t i = 0; i < k; ++i) {
      GR_TRY(gr_sssp(ctx, g, sources + i, 1, dist + (int64_t)i * V,
                     pred ? pred + (int64_t)i * V : nullptr, &o1, stream, &s1));
      agg.iterations = std::max(agg.iterations, s1.iterations);
      for (int a = 0; a < 4; ++a) agg.action_count[a] += s1.action_count[a];
      agg.teps_edges += s1.teps_edges;
      agg.inspected_edges += s1.inspected_edges;
      agg.device_ms += s1.device_ms;
    }
    if (stats) *stats = agg;
    return GR_OK;
  }
  const int chunk = msssp_chunk(opts.lb_chunk > 0 ? opts.lb_chunk : 1024);
  constexpr int kPass = 16;
  const int KSmax = msssp_row(std::min<int32_t>(k, kPass));

  unsigned long long* keys;
  uint32_t *amask, *nmask, *fmask = nullptr;
  int32_t *qA, *qB, *qC, *offsets, *rstart, *chunks, *src_dev, *piles = nullptr;
  int64_t* bsums;
  Ctrl* ctrl;
  GR_TRY(pool_typed(ctx, S_MS_KEYS, (size_t)V * KSmax, &keys));
  uint32_t* relaxed = nullptr;
  if (!(opts.sssp_opt_off & GR_SSSP_OPT_CULL))
    GR_TRY(pool_typed(ctx, S_MS_RELAXED, (size_t)V * KSmax, &relaxed));
  GR_TRY(pool_typed(ctx, S_MS_AMASK, V, &amask));
  GR_TRY(pool_typed(ctx, S_MS_NMASK, V, &nmask));
  // near / far split (sssp_delta > 0): far-pair masks and two far piles
  const bool use_pq = opts.sssp_delta > 0;
  GR_TRY(pool_typed(ctx, S_MS_FMASK, V, &fmask));
  if (use_pq) GR_TRY(pool_typed(ctx, S_FAR, 2 * (size_t)V, &piles));
  GR_TRY(pool_typed(ctx, S_Q_A, V, &qA));
  GR_TRY(pool_typed(ctx, S_Q_B, V, &qB));
  GR_TRY(pool_typed(ctx, S_Q_C, V, &qC));
  GR_TRY(pool_typed(ctx, S_OFFSETS, V + 1, &offsets));
  GR_TRY(pool_typed(ctx, S_RSTART, V, &rstart));
  GR_TRY(pool_typed(ctx, S_CHUNKS, E / 512 + 2, &chunks));
  GR_TRY(pool_typed(ctx, S_BLOCK_SUMS, stats_grid() + 1, &bsums));
  GR_TRY(pool_typed(ctx, S_CTRL, 1, &ctrl));
  GR_TRY(pool_typed(ctx, S_TMP0, 2 * kPass, &src_dev));
  Ctrl* hc = ctx->host_ctrl;
  // q[cur]: the frontier; relax appends the improved vertices to q[cur + 1],
  // rotate lists those with an active source left in q[cur + 2], the next
  // frontier (queue indices mod 3)
  int32_t* q[3] = {qA, qB, qC};

  GR_HIP(hipEventRecord(ctx->ev_start, st));
  GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->reached_edges), 2, 0u, st));
  gr_run_stats rs{};
  int max_it = 0;
  std::vector<int32_t> srcs, uniq;
  for (int32_t p0 = 0; p0 < k; p0 += kPass) {
    const int32_t kk = std::min<int32_t>(kPass, k - p0);
    const int KS = msssp_row(kk);
    // src_dev: the pass's sources in traversal ids, then in caller ids
    srcs.resize(2 * (size_t)kk);
    for (int32_t i = 0; i < kk; ++i) {
      srcs[i] = g->to_new(sources[p0 + i]);
      srcs[kk + i] = sources[p0 + i];
    }
    uniq.assign(srcs.begin(), srcs.begin() + kk);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    GR_HIP(hipMemcpyAsync(src_dev, srcs.data(), sizeof(int32_t) * 2 * kk, hipMemcpyHostToDevice, st));
    GR_HIP(hipMemcpyAsync(qA, uniq.data(), sizeof(int32_t) * uniq.size(), hipMemcpyHostToDevice, st));
    GR_HIP(launch_fill_u32(&ctrl->q_count[0], 1, (uint32_t)uniq.size(), st));
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->m_f[0]), 8, 0u, st));  // m_f, max_deg
    GR_HIP(launch_msssp_init(keys, KS, amask, nmask, fmask, relaxed, V, src_dev, kk, st));
    GR_HIP(launch_fill_u32(&ctrl->far_count[0], 2, 0u, st));
    int cur = 0, sp = 0, it = 0, pile = 0;
    uint32_t T = (uint32_t)opts.sssp_delta;
    GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                 &ctrl->q_count[(cur + 1) % 3], &ctrl->q_count[(cur + 2) % 3], st));
    GR_TRY(read_ctrl(ctx, ctrl, st));  // also keeps the host source vectors alive for the copies
    int64_t n_f = hc->n_f[sp], m_f = hc->m_f[sp], far_n = 0;
    while ((n_f > 0 || far_n > 0) && (opts.max_iterations <= 0 || it < opts.max_iterations)) {
      if (n_f == 0) {
        // the frontier ran dry: raise the threshold and split the far pile
        // into the frontier (appended to the empty queue q[cur])
        const uint64_t t1 = (uint64_t)T + (uint64_t)opts.sssp_delta;
        const uint32_t T1 = t1 >= 0xffffffffull ? 0xffffffffu : (uint32_t)t1;
        GR_HIP(launch_fill_u32(&ctrl->far_count[pile ^ 1], 1, 0u, st));
        GR_HIP(launch_msssp_refill(piles + (int64_t)pile * V, &ctrl->far_count[pile], far_n,
                                   piles + (int64_t)(pile ^ 1) * V, &ctrl->far_count[pile ^ 1], keys,
                                   KS, fmask, amask, T, T1, q[cur], &ctrl->q_count[cur], st));
        T = T1;
        pile ^= 1;
      } else {
        GR_HIP(launch_frontier_offsets(q[cur], n_f, g->R, bsums, &ctrl->m_f[sp], offsets, rstart,
                                       chunks, chunk, st));
        const MsFar far{fmask, use_pq ? piles + (int64_t)pile * V : nullptr, &ctrl->far_count[pile],
                        T};
        const int q1 = (cur + 1) % 3, q2 = (cur + 2) % 3;
        GR_HIP(launch_msssp_relax(KS, chunk, q[cur], offsets, rstart, chunks, n_f, m_f, g->C, g->W,
                                  keys, amask, nmask, use_pq ? &far : nullptr, g->perm, relaxed,
                                  q[q1], &ctrl->q_count[q1], st));
        GR_HIP(launch_msssp_rotate(q[cur], &ctrl->q_count[cur], n_f, q[q1], &ctrl->q_count[q1],
                                   std::min<int64_t>(V, m_f), amask, nmask, keys, KS, relaxed,
                                   q[q2], &ctrl->q_count[q2], st));
        rs.inspected_edges += m_f;
        rs.action_count[GR_PUSH_LB]++;
        cur = q2;
        sp ^= 1;
      }
      ++it;
      GR_HIP(launch_frontier_stats(q[cur], &ctrl->q_count[cur], g->R, bsums, ctrl, sp,
                                   &ctrl->q_count[(cur + 1) % 3], &ctrl->q_count[(cur + 2) % 3],
                                   st));
      GR_TRY(read_ctrl(ctx, ctrl, st));
      n_f = hc->n_f[sp];
      m_f = hc->m_f[sp];
      far_n = use_pq ? hc->far_count[pile] : 0;
    }
    max_it = std::max(max_it, it);
    GR_HIP(launch_msssp_finalize(keys, KS, kk, g->R, V, dist + (int64_t)p0 * V,
                                 pred ? pred + (int64_t)p0 * V : nullptr, g->perm, src_dev + kk,
                                 &ctrl->reached_edges, st));
  }
  GR_HIP(hipEventRecord(ctx->ev_stop, st));
  GR_TRY(read_ctrl(ctx, ctrl, st));
  if (stats) {
    float ms = 0.f;
    GR_TRY(elapsed_ms(ctx->ev_start, ctx->ev_stop, &ms));
    rs.iterations = max_it;
    rs.teps_edges = hc->reached_edges;
    rs.device_ms = ms;
    *stats = rs;
  }
  return GR_OK;
}

// ============================================================================
// betweenness centrality (Sec. 6, Brandes's forward and backward passes)
// ============================================================================

extern "C" gr_status gr_bc(gr_ctx* ctx, const gr_graph* g, const int32_t* sources,
                           int32_t n_sources, double* bc, double* sigma, gr_opts* opts_in,
                           void* stream, gr_run_stats* stats) {
  if (!ctx || !g) return fail(GR_EINVAL, "gr_bc: ctx or graph is NULL");
  if (g->ctx != ctx) return fail(GR_EINVAL, "gr_bc: graph belongs to another context");
  if (!bc) return fail(GR_EINVAL, "gr_bc: bc is NULL");
  if (!sources || n_sources < 1) return fail(GR_EINVAL, "gr_bc: need at least one source");
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || (int64_t)sources[i] >= g->V)
      return fail(GR_EINVAL, "gr_bc: source " + std::to_string(sources[i]) + " out of range");
  if (sigma && n_sources != 1) return fail(GR_EINVAL, "gr_bc: sigma needs exactly one source");
  if (!(g->flags & GR_SYMMETRIC))
    return fail(GR_EUNSUPPORTED, "gr_bc needs a symmetric graph (each pass follows edges against their direction)");
  gr_opts opts;
  GR_TRY(check_opts(opts_in, &opts));
  if (opts_in) opts_in->trace_count = 0;
  opts.trace = nullptr;       // the BFS inside is not traced
  opts.trace_capacity = 0;
  opts.max_iterations = 0;    // every level is needed
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t V = g->V, E = g->E;
  const AdvCfg adv = adv_cfg(opts);
  const int chunk = adv.chunk;
  const bool lb = (double)E / (double)V >= (double)opts.lb_min_avg_degree;
  const int dir_sigma = opts.bc_dir & 3, dir_dep = opts.bc_dir >> 2;
  // push when forced, or (auto) when the level the sums come from has under
  // 1 / kBcPushBias of the edges of the level they belong to and under
  // kBcPushFanIn edges per vertex of that level: a pushed edge costs about
  // what a pulled one does until many of them add into the same few
  // vertices, whose fp64 atomics then queue one behind another
  constexpr unsigned long long kBcPushBias = 4, kBcPushFanIn = 64;
  auto use_push = [](int dir, unsigned long long m_from, unsigned long long m_to,
                     unsigned long long n_to) {
    if (dir != GR_BC_DIR_AUTO) return dir == GR_BC_DIR_PUSH;
    return m_from * kBcPushBias < m_to && m_from < n_to * kBcPushFanIn;
  };

  int32_t *depth, *levels, *chunks, *all_offs, *all_rstart;
  double *sig, *acc;
  uint32_t* lvl_n;
  unsigned long long* lvl_m;
  int64_t* bsums;
  Ctrl* ctrl;
  GR_TRY(pool_typed(ctx, S_BC_DEPTH, V, &depth));
  GR_TRY(pool_typed(ctx, S_BC_SIGMA, V, &sig));
  GR_TRY(pool_typed(ctx, S_BC_ACC, V, &acc));
  GR_TRY(pool_typed(ctx, S_BC_LEVELS, V, &levels));
  GR_TRY(pool_typed(ctx, S_BC_LVL_N, 2 * (size_t)(V + 1), &lvl_n));  // counts, then cursors
  GR_TRY(pool_typed(ctx, S_BC_LVL_M, V + 1, &lvl_m));
  // degree scan and row starts of all levels' vertices (level order)
  GR_TRY(pool_typed(ctx, S_OFFSETS, V + 1, &all_offs));
  GR_TRY(pool_typed(ctx, S_RSTART, V, &all_rstart));
  GR_TRY(pool_typed(ctx, S_CHUNKS, E / 512 + 2, &chunks));
  GR_TRY(pool_typed(ctx, S_BLOCK_SUMS, stats_grid() + 1, &bsums));
  GR_TRY(pool_typed(ctx, S_CTRL, 1, &ctrl));

  GR_HIP(hipEventRecord(ctx->ev_c0, st));
  GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(bc), 2 * V, 0u, st));
  Arena ar;
  ar.ctx = ctx;
  gr_run_stats rs{};
  std::vector<uint32_t> hn;
  std::vector<unsigned long long> hm;
  std::vector<uint32_t> off;
  std::vector<int64_t> tab;
  int sp = 0;
  for (int32_t i = 0; i < n_sources; ++i) {
    gr_run_stats bs{};
    GR_TRY(bfs_run(ctx, g, sources[i], depth, nullptr, nullptr, opts, st, &bs, ar,
                   /*internal_ids=*/true));
    const int32_t L = bs.iterations;  // levels 0 .. L - 1 are non-empty
    const int32_t src = g->to_new(sources[i]);
    GR_HIP(launch_fill_u32(lvl_n, L, 0u, st));
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(lvl_m), 2 * (int64_t)L, 0u, st));
    GR_HIP(launch_bc_levels(depth, g->R, V, src, L, lvl_n, lvl_m, sig, acc, st));
    hn.resize(L);
    hm.resize(L);
    off.assign((size_t)L + 1, 0u);
    GR_HIP(hipMemcpyAsync(hn.data(), lvl_n, sizeof(uint32_t) * L, hipMemcpyDeviceToHost, st));
    GR_HIP(hipMemcpyAsync(hm.data(), lvl_m, sizeof(unsigned long long) * L, hipMemcpyDeviceToHost,
                          st));
    GR_HIP(hipStreamSynchronize(st));
    // per level: first vertex index, first edge position and first chunk of
    // the pull passes' maps (levels stored one after another)
    tab.assign(3 * (size_t)L, 0);
    for (int32_t d = 0; d < L; ++d) {
      off[d + 1] = off[d] + hn[d];
      tab[d] = off[d];
      if (d + 1 < L) {
        tab[L + d + 1] = tab[L + d] + (int64_t)hm[d];
        tab[2 * L + d + 1] = tab[2 * L + d] + ((int64_t)hm[d] + chunk - 1) / chunk;
      }
    }
    const int64_t n_r = off[L];
    const int64_t n_chunks = tab[2 * L + L - 1] + ((int64_t)hm[L - 1] + chunk - 1) / chunk;
    int64_t* tab_dev;
    int32_t* bc_chunks;
    GR_TRY(pool_typed(ctx, S_BC_TAB, tab.size(), &tab_dev));
    GR_TRY(pool_typed(ctx, S_BC_CHUNKS, (size_t)n_chunks + 1, &bc_chunks));
    GR_HIP(hipMemcpyAsync(lvl_n + L, off.data(), sizeof(uint32_t) * L, hipMemcpyHostToDevice, st));
    GR_HIP(hipMemcpyAsync(tab_dev, tab.data(), sizeof(int64_t) * tab.size(), hipMemcpyHostToDevice,
                          st));
    GR_HIP(launch_bc_scatter(depth, V, L, lvl_n + L, levels, st));
    GR_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(&ctrl->m_f[0]), 8, 0u, st));  // m_f, max_deg
    sp = 0;
    // the LB maps of all levels at once: one degree scan over the reached
    // vertices in level order (its chunk output is not used: the chunk size
    // given puts every edge in chunk 0 or 1), then every level's chunk map
    // (the last level's cursor ends at n_r)
    GR_HIP(launch_frontier_stats(levels, lvl_n + L + L - 1, g->R, bsums, ctrl, sp, nullptr, nullptr,
                                 st));
    GR_HIP(launch_frontier_offsets(levels, n_r, g->R, bsums, &ctrl->m_f[sp], all_offs, all_rstart,
                                   chunks, 1 << 30, st));
    sp ^= 1;
    GR_HIP(launch_bc_chunk_map(levels, depth, n_r, all_offs, tab_dev, L, chunk, bc_chunks, st));
    // one pass over level x's rows (edges into depth `want`): pulled, or
    // pushed over LB chunks (TWC where the average degree is below
    // lb_min_avg_degree)
    auto sweep_level = [&](bool dependency, bool push, int32_t x, int32_t want) -> hipError_t {
      const int32_t* f = levels + off[x];
      const int32_t* o = all_offs + off[x];
      const int32_t* r = all_rstart + off[x];
      const int32_t* cm = bc_chunks + tab[2 * L + x];
      if (!push)
        return launch_bc_pull(dependency, f, o, r, cm, hn[x], (int64_t)hm[x], tab[L + x], chunk,
                              g->C, depth, want, sig, acc, st);
      const int mode = lb ? 2 : 0;
      if (dependency)
        return launch_bc_dependency(mode, f, o, r, cm, hn[x], (int64_t)hm[x], tab[L + x], g->R,
                                    g->C, depth, sig, acc, want, adv, st);
      return launch_bc_sigma(mode, f, o, r, cm, hn[x], (int64_t)hm[x], tab[L + x], g->R, g->C,
                             depth, sig, want, adv, st);
    };
    // forward: sigma of level d + 1 from level d, pushed by level d or
    // gathered by level d + 1
    for (int32_t d = 0; d + 1 < L; ++d) {
      const bool push = use_push(dir_sigma, hm[d], hm[d + 1], hn[d + 1]);
      const int32_t x = push ? d : d + 1;  // the level whose rows are swept
      if (hm[x] == 0) continue;
      GR_HIP(sweep_level(false, push, x, push ? d + 1 : d));
    }
    // backward: dependency sums of level d - 1 from level d, pushed by level d
    // or gathered by level d - 1 (the source's own sum is not needed)
    for (int32_t d = L - 1; d >= 2; --d) {
      const bool push = use_push(dir_dep, hm[d], hm[d - 1], hn[d - 1]);
      const int32_t x = push ? d : d - 1;
      if (hm[x] == 0) continue;
      GR_HIP(sweep_level(true, push, x, push ? d - 1 : d));
    }
    GR_HIP(launch_bc_finalize(depth, sig, acc, V, src, g->perm, bc, sigma, st));
    // the host vectors are reused by the next source: finish their copies
    GR_HIP(hipStreamSynchronize(st));
    rs.iterations += L;
    rs.teps_edges += bs.teps_edges;
    rs.inspected_edges += bs.inspected_edges;
    for (int a = 0; a < 4; ++a) rs.action_count[a] += bs.action_count[a];
  }
  GR_HIP(hipEventRecord(ctx->ev_c1, st));
  GR_HIP(hipEventSynchronize(ctx->ev_c1));
  if (stats) {
    float ms = 0.f;
    GR_TRY(elapsed_ms(ctx->ev_c0, ctx->ev_c1, &ms));
    rs.device_ms = ms;
    *stats = rs;
  }
  return GR_OK;
}

extern "C" gr_status gr_ctx_set_policy(gr_ctx* ctx, const float* params, int32_t n_params) {
  if (!ctx) return fail(GR_EINVAL, "gr_ctx_set_policy: ctx is NULL");
  if (!params) {
    ctx->policy_loaded = false;
    ctx->mlp_multi_offset = 0;
    return GR_OK;
  }
  if (n_params != GR_MLP_N_PARAMS && n_params != 2 * GR_MLP_N_PARAMS)
    return fail(GR_EINVAL, "gr_ctx_set_policy: expected " + std::to_string(GR_MLP_N_PARAMS) +
                               " or " + std::to_string(2 * GR_MLP_N_PARAMS) + " parameters, got " +
                               std::to_string(n_params));
  for (int32_t i = 0; i < n_params; ++i)
    if (!std::isfinite(params[i])) return fail(GR_EINVAL, "gr_ctx_set_policy: non-finite parameter");
  DeviceGuard dg(ctx->device);
  float* d = nullptr;
  GR_TRY(pool_typed(ctx, S_MLP, 2 * (size_t)GR_MLP_N_PARAMS, &d));
  GR_HIP(hipMemcpy(d, params, sizeof(float) * n_params, hipMemcpyHostToDevice));
  ctx->policy_loaded = true;
  ctx->mlp_multi_offset = n_params == 2 * GR_MLP_N_PARAMS ? GR_MLP_N_PARAMS : 0;
  return GR_OK;
}

// ============================================================================
// selector network training / inference (device buffers)
// ============================================================================

extern "C" gr_status gr_mlp_forward(gr_ctx* ctx, const float* params, const float* X, int32_t n,
                                    float* Y, void* stream) {
  if (!ctx || !params || (n > 0 && (!X || !Y))) return fail(GR_EINVAL, "gr_mlp_forward: NULL argument");
  if (n < 0) return fail(GR_EINVAL, "gr_mlp_forward: n < 0");
  DeviceGuard dg(ctx->device);
  GR_HIP(launch_mlp_forward(params, X, n, Y, static_cast<hipStream_t>(stream)));
  return GR_OK;
}

extern "C" gr_status gr_mlp_loss_grad(gr_ctx* ctx, const float* params, const float* X,
                                      const float* T, const float* M, int32_t n, float* grad,
                                      float* loss, void* stream) {
  if (!ctx || !params || !grad || (n > 0 && (!X || !T || !M)))
    return fail(GR_EINVAL, "gr_mlp_loss_grad: NULL argument");
  if (n < 0) return fail(GR_EINVAL, "gr_mlp_loss_grad: n < 0");
  DeviceGuard dg(ctx->device);
  const int64_t tiles = (std::max<int64_t>(n, 1) + mlp_tile() - 1) / mlp_tile();
  float* partial = nullptr;
  GR_TRY(pool_typed(ctx, S_MLP_WS, (size_t)tiles * (GR_MLP_N_PARAMS + 2), &partial));
  GR_HIP(launch_mlp_loss_grad(params, X, T, M, n, partial, grad, loss,
                              static_cast<hipStream_t>(stream)));
  return GR_OK;
}

extern "C" gr_status gr_mlp_adam(gr_ctx* ctx, float* params, const float* grad, float* m, float* v,
                                 int32_t step, float lr, float beta1, float beta2, float eps,
                                 void* stream) {
  if (!ctx || !params || !grad || !m || !v) return fail(GR_EINVAL, "gr_mlp_adam: NULL argument");
  if (step < 1) return fail(GR_EINVAL, "gr_mlp_adam: step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr > 0.f))
    return fail(GR_EINVAL, "gr_mlp_adam: need lr > 0, 0 <= beta < 1, eps > 0");
  DeviceGuard dg(ctx->device);
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  GR_HIP(launch_adam(params, grad, m, v, GR_MLP_N_PARAMS, lr, beta1, beta2, eps, c1, c2,
                     static_cast<hipStream_t>(stream)));
  return GR_OK;
}

// ============================================================================
// measurement
// ============================================================================

extern "C" gr_status gr_copy_bandwidth(gr_ctx* ctx, int64_t bytes, int32_t reps, void* stream,
                                       float* gbps) {
  if (!ctx || !gbps) return fail(GR_EINVAL, "gr_copy_bandwidth: NULL argument");
  if (bytes <= 0 || bytes % 16 != 0) return fail(GR_EINVAL, "bytes must be a positive multiple of 16");
  if (reps < 1) return fail(GR_EINVAL, "reps must be >= 1");
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  void *a = nullptr, *b = nullptr;
  GR_HIP(hipMalloc(&a, (size_t)bytes));
  hipError_t e = hipMalloc(&b, (size_t)bytes);
  if (e != hipSuccess) {
    (void)hipFree(a);
    return fail(GR_ENOMEM, "gr_copy_bandwidth: allocation failed");
  }
  struct Free2 {
    void *x, *y;
    ~Free2() {
      (void)hipFree(x);
      (void)hipFree(y);
    }
  } fr{a, b};
  GR_HIP(launch_fill_u32(static_cast<uint32_t*>(a), bytes / 4, 1u, st));
  GR_HIP(launch_copy(a, b, bytes, st));
  GR_HIP(hipEventRecord(ctx->ev_k0, st));
  for (int i = 0; i < reps; ++i) GR_HIP(launch_copy(a, b, bytes, st));
  GR_HIP(hipEventRecord(ctx->ev_k1, st));
  GR_HIP(hipEventSynchronize(ctx->ev_k1));
  float ms = 0.f;
  GR_TRY(elapsed_ms(ctx->ev_k0, ctx->ev_k1, &ms));
  *gbps = (float)(2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9);
  return GR_OK;
}
