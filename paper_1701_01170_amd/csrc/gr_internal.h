// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "gr.h"

namespace gr {

// ---- error reporting ------------------------------------------------------

void set_error(const std::string& msg);
gr_status fail(gr_status code, const std::string& msg);

#define GR_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess)                                                              \
      return ::gr::fail(_e == hipErrorOutOfMemory ? GR_ENOMEM : GR_EHIP,               \
                        std::string(#call) + ": " + hipGetErrorString(_e));            \
  } while (0)

#define GR_TRY(expr)                   \
  do {                                 \
    gr_status _s = (expr);             \
    if (_s != GR_OK) return _s;        \
  } while (0)

// ---- pooled device scratch ---------------------------------------------------

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Slots of the per-context scratch pool.
enum Slot : int {
  S_BM_A = 0,      // visited bitmap (ping)
  S_BM_B,          // visited bitmap (pong)
  S_Q_A,           // vertex frontier queue (ping)
  S_Q_B,           // vertex frontier queue (pong)
  S_U_A,           // unvisited frontier (ping)
  S_U_B,           // unvisited frontier (pong)
  S_OFFSETS,       // exclusive scan of frontier degrees [n_f + 1]
  S_BLOCK_SUMS,    // per-block partial sums/max for the frontier scan
  S_CTRL,          // device control block (counters and level statistics)
  S_KEYS,          // SSSP packed (dist << 32 | pred) keys [V]
  S_TAGS,          // SSSP output-queue tags [V]
  S_MASK_A,        // multi-source masks
  S_MASK_B,
  S_MASK_C,
  S_MLP,           // selector parameters on the device
  S_TMP0,
  S_TMP1,
  S_NSLOTS
};

// Device control block.  Counters used for appends are 32-bit; sums are 64-bit.
struct Ctrl {
  uint32_t q_count[2];      // frontier queue lengths (ping/pong)
  uint32_t u_count[2];      // unvisited frontier lengths (ping/pong)
  int64_t m_f;              // sum of frontier degrees
  int64_t max_deg;          // largest frontier degree
  int64_t n_f;              // frontier size as seen by the statistics kernel
  int64_t inspected;        // pull: neighbours scanned (accumulated)
  int32_t action;           // action chosen on the device (learned policy)
  int32_t pad0;
  int64_t reached_edges;    // sum of degrees over reached vertices (end of run)
  int64_t misc[4];
};

}  // namespace gr

struct gr_ctx {
  int device = 0;
  int cu_count = 256;
  gr::DevBuf pool[gr::S_NSLOTS];
  gr::Ctrl* host_ctrl = nullptr;   // pinned host mirror of the control block
  bool policy_loaded = false;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_a = nullptr, ev_b = nullptr;
};

struct gr_graph {
  gr_ctx* ctx = nullptr;
  int64_t V = 0, E = 0;
  int64_t max_degree = 0;
  uint32_t flags = 0;
  uint32_t max_weight = 0;
  int32_t resorted = 0;
  int32_t* R = nullptr;   // device row offsets [V+1]
  int32_t* C = nullptr;   // device column indices [E], each row ascending
  uint32_t* W = nullptr;  // device weights [E] or null
};

namespace gr {

gr_status pool_get(gr_ctx* ctx, Slot s, size_t bytes, void** out);

// ---- kernel launchers (defined in the .hip files) -----------------------------

// ingest
hipError_t launch_csr_check(const int32_t* R, const int32_t* C, int64_t V, int64_t E,
                            int64_t* flags_dev, hipStream_t st);
hipError_t launch_row_sort(int32_t* R, int32_t* C, uint32_t* W, int64_t V, const int32_t* rows,
                           int64_t n_rows, uint64_t* scratch, hipStream_t st);
hipError_t launch_find_unsorted(const int32_t* R, const int32_t* C, const uint32_t* W, int64_t V,
                                int32_t* rows_out, uint32_t* count, hipStream_t st);
hipError_t launch_graph_stats(const int32_t* R, const uint32_t* W, int64_t V, int64_t E,
                              int64_t* out2, hipStream_t st);

// frontier statistics and scan
int stats_grid();
hipError_t launch_frontier_stats(const int32_t* frontier, const uint32_t* n_f_dev, const int32_t* R,
                                 int64_t* block_sums, Ctrl* ctrl, uint32_t* zero_a,
                                 uint32_t* zero_b, hipStream_t st);
hipError_t launch_frontier_offsets(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                   const int64_t* block_sums, int32_t* offsets,
                                   uint32_t* live_bm, hipStream_t st);

// BFS
hipError_t launch_bfs_init(int32_t* depth, int32_t* parent, int64_t V, uint32_t* bm_old,
                           uint32_t* bm_live, int64_t n_words, int32_t source, int32_t* queue,
                           Ctrl* ctrl, hipStream_t st);
hipError_t launch_bfs_push_lb(const int32_t* frontier, const int32_t* offsets, int64_t n_f,
                              int64_t m_f, const int32_t* R, const int32_t* C,
                              const uint32_t* bm_old, uint32_t* bm_live, int32_t* depth,
                              int32_t* parent, int32_t next_depth, int32_t* out_q,
                              uint32_t* out_count, int chunk, hipStream_t st);
hipError_t launch_bfs_push_light(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                 const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                                 int32_t* depth, int32_t* parent, int32_t next_depth,
                                 int32_t* out_q, uint32_t* out_count, hipStream_t st);
hipError_t launch_bfs_push_twc(const int32_t* frontier, int64_t n_f, const int32_t* R,
                               const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                               int32_t* depth, int32_t* parent, int32_t next_depth,
                               int32_t* out_q, uint32_t* out_count, hipStream_t st);
hipError_t launch_gen_unvisited(const uint32_t* bm_old, const int32_t* R, int64_t V,
                                int32_t* out_list, uint32_t* out_count, hipStream_t st);
hipError_t launch_bfs_pull(bool lb, const int32_t* unvisited, int64_t n_u, const int32_t* R,
                           const int32_t* C, const uint32_t* bm_old, uint32_t* bm_live,
                           int32_t* depth, int32_t* parent, int32_t next_depth,
                           int32_t* out_active, uint32_t* out_active_count,
                           int32_t* out_unvisited, uint32_t* out_unvisited_count,
                           int64_t* inspected, hipStream_t st);
hipError_t launch_bitmap_or(uint32_t* dst, const uint32_t* src, int64_t n_words, hipStream_t st);
hipError_t launch_reached_edges(const int32_t* depth, const int32_t* R, int64_t V, int64_t* out,
                                hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st);

// SSSP
hipError_t launch_sssp_init(unsigned long long* keys, int32_t* tags, int64_t V, Ctrl* ctrl,
                            hipStream_t st);
hipError_t launch_sssp_seed(const int32_t* src_dev, int32_t n, unsigned long long* keys,
                            int32_t* tags, Ctrl* ctrl, hipStream_t st);
hipError_t launch_sssp_relax(int action_lb, bool light, const int32_t* frontier,
                             const int32_t* offsets, int64_t n_f, int64_t m_f, const int32_t* R,
                             const int32_t* C, const uint32_t* W, unsigned long long* keys,
                             int32_t* tags, int32_t next_tag, int32_t* out_q, uint32_t* out_count,
                             int chunk, hipStream_t st);
hipError_t launch_sssp_finalize(const unsigned long long* keys, const int32_t* R, int64_t V,
                                uint32_t* dist, int32_t* pred, const int32_t* src_dev,
                                int32_t n_src, int64_t* reached_edges, hipStream_t st);

}  // namespace gr
