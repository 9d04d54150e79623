// Internal declarations shared by the host runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <vector>
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
  S_BM = 0,        // visited bitmaps, interleaved word pairs (old/live)
  S_Q_A,           // vertex frontier queue (ping)
  S_Q_B,           // vertex frontier queue (second)
  S_Q_C,           // vertex frontier queue (third; device-predicated levels rotate three)
  S_DLOG,          // per-level log of a device-predicated block (n_f, m_f, max degree)
  S_FAR,           // SSSP far piles: three rotating int32[V]
  S_FAR_TAGS,      // SSSP far-pile generation per vertex
  S_DEPTH,         // BFS depth / parent in renumbered ids (mapped back at the end)
  S_PARENT,
  S_OFFSETS,       // exclusive scan of frontier degrees [n_f + 1]
  S_RSTART,        // row start of every frontier vertex [n_f]
  S_BLOCK_SUMS,    // per-block partial sums for the frontier scan
  S_CTRL,          // device control block (counters and level statistics)
  S_KEYS,          // shortest-path packed (dist << 32 | pred) keys [V]
  S_TAGS,          // shortest-path output-queue tags [V]
  S_MASK_A,        // multi-source masks
  S_MASK_B,
  S_MASK_C,
  S_MLP,           // selector parameters on the device
  S_TMP0,          // small per-call staging (source lists)
  S_CHUNKS,        // LB chunk -> first frontier segment map
  S_MARKS,         // one byte per vertex, all zero between uses
  S_MLP_WS,        // selector gradient partial sums
  S_MIRROR,        // shortest-path one-byte distance mirror [V]
  S_RELAXED,       // shortest-path: 1 + distance a frontier vertex's edges were relaxed with [V]
  S_SSSP_BINS,     // shortest-path distance bins: histograms, cursors, base
  S_MS_RELAXED,    // batched shortest paths: per (vertex, source) cull values [V * row]
  S_UL_A,          // BFS pull: unvisited vertices with neighbours (two lists, ping-pong)
  S_UL_B,
  S_CAND,          // BFS idempotent advance: candidate list [V]
  S_BC_DEPTH,      // betweenness centrality: depths from the current source [V]
  S_BC_SIGMA,      // shortest-path counts [V] (double)
  S_BC_ACC,        // dependency sums [V] (double)
  S_BC_LEVELS,     // vertices grouped by level [V]
  S_BC_LVL_N,      // vertices per level, then level cursors [L + 1]
  S_BC_LVL_M,      // degree sum per level [L + 1]
  S_BC_CHUNKS,     // per-level LB chunk -> first-row maps, level after level (the
                   // levels' degree scan and row starts use S_OFFSETS / S_RSTART)
  S_BC_TAB,        // per level: first vertex index, first edge position, first chunk [3 L]
  S_MS_KEYS,       // batched SSSP: packed keys, KS per vertex [V * KS]
  S_MS_AMASK,      // batched SSSP: sources a frontier vertex is active for [V]
  S_MS_NMASK,      // batched SSSP: sources whose distance dropped this iteration [V]
  S_MS_FMASK,      // batched SSSP: pairs waiting on the far pile [V]
  S_NSLOTS
};

// Device control block.  Counters used for appends are 32-bit; sums are
// 64-bit.  Frontier statistics use two slots selected by the parity of the
// statistics call, so each call can clear the slot the next one accumulates in.
struct Ctrl {
  uint32_t q_count[3];      // frontier queue lengths (three rotating queues)
  uint32_t cand_count;      // BFS idempotent advance: candidate list length (may exceed its capacity)
  int64_t m_f[2];           // sum of frontier degrees
  int64_t max_deg[2];       // largest frontier degree
  int64_t n_f[2];           // frontier size as seen by the statistics kernel
  int64_t inspected;        // pull: neighbours scanned (accumulated)
  int64_t reached_edges;    // sum of degrees over reached vertices (end of run)
  int32_t action;           // network argmin over the allowed actions (learned policy)
  float pred[4];            // the network's predicted log2 step times (disallowed: +inf)
  int32_t pad0;
  uint32_t ul_count[2];     // BFS pull: lengths of the two unvisited lists
  uint32_t pad3[6];
  // device-predicated level blocks (iteration control without host round trips)
  int32_t dl_levels;        // levels of the current block that ran
  int32_t dl_stop;          // a level of the block declined to run
  int64_t dl_vm[2];         // degree sum of the vertices reached before the current frontier
  int64_t dl_vn[2];         // number of vertices reached before the current frontier
  // SSSP two-level priority queue (near / far piles); [2] slots alternate by
  // level inside a device-predicated block
  uint32_t pq_T[2];         // near threshold
  int32_t pq_epoch[2];      // far-pile generation (dedups far appends)
  int32_t pq_fc[2];         // far pile in use (of three rotating piles)
  uint32_t far_count[3];    // far pile lengths
  uint32_t pad2;
  // multi-source BFS: (source, vertex) pairs reached so far and the sum of
  // their degrees (the selector's unvisited counts, averaged over sources)
  int64_t ms_pairs;
  int64_t ms_pair_edges;
};

}  // namespace gr

struct gr_ctx {
  int device = 0;
  int cu_count = 256;
  gr::DevBuf pool[gr::S_NSLOTS];
  // Host view of the control block: coherent pinned host memory that a small
  // kernel fills (followed by a sequence number in publish_flag) after each
  // step, so the host polls memory instead of synchronising the stream.
  gr::Ctrl* host_ctrl = nullptr;
  gr::Ctrl* host_ctrl_dev = nullptr;        // the same memory, device address
  volatile uint32_t* publish_flag = nullptr;
  uint32_t* publish_flag_dev = nullptr;
  // a device-predicated block's level log (3 x kDlMaxLevels int64), copied
  // here by the publication that ends the block while tracing
  int64_t* host_dlog = nullptr;
  int64_t* host_dlog_dev = nullptr;
  uint32_t publish_seq = 0;
  bool policy_loaded = false;
  // offset of the batched-traversal network in the selector parameters (0:
  // the same network serves every traversal)
  int32_t mlp_multi_offset = 0;
  // Device address of this device's copy of the library's static workspace
  // (gr_bfs_static), looked up once per device when the context is created.
  void* static_ws = nullptr;
  // Longest wait for one published control block before a traversal gives up
  // with GR_EHIP (environment GR_WAIT_LIMIT_MS at context creation, default 60 s).
  std::chrono::milliseconds wait_limit{60000};
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_a = nullptr, ev_b = nullptr;
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;  // around the advance kernel when tracing
  hipEvent_t ev_c0 = nullptr, ev_c1 = nullptr;  // around a whole call that runs BFS inside
  // hipGraph iteration control (gr_opts.graph_blocks): a stream nothing runs
  // on, used only to capture the launches of a block of device-predicated
  // levels, and the instantiated graph per block shape (traversal, length).
  hipStream_t cap_stream = nullptr;
  std::map<int, hipGraphExec_t> block_graphs;
};

struct gr_graph {
  gr_ctx* ctx = nullptr;
  int64_t V = 0, E = 0;
  int64_t max_degree = 0;
  uint32_t flags = 0;
  uint32_t max_weight = 0;
  int32_t resorted = 0;
  // Traversals run on the CSR below.  With GR_RENUMBER its vertices are
  // renumbered by descending degree (ties by id): row i is the
  // caller's row perm[i] with every neighbour renamed and kept in the
  // caller's order (ascending original ids), so "first frontier neighbour"
  // is still the smallest original id.  Outputs are mapped back.
  int32_t* R = nullptr;   // device row offsets [V+1]
  int32_t* C = nullptr;   // device column indices [E]
  uint32_t* W = nullptr;  // device weights [E] or null
  int32_t* perm = nullptr;    // new id -> caller id (null: ids kept)
  int32_t* inv = nullptr;     // caller id -> new id
  int32_t* R_orig = nullptr;  // caller's row offsets (export)
  std::vector<int32_t> inv_host;  // caller id -> new id, for host-given sources
  int32_t to_new(int32_t v) const { return perm ? inv_host[(size_t)v] : v; }
};

namespace gr {

gr_status pool_get(gr_ctx* ctx, Slot s, size_t bytes, void** out);

// Launch shape of the push-advance kernels (tuning knobs: the results never
// depend on them).
struct AdvCfg {
  int chunk = 8192;         // LB: edges per workgroup (512 .. 16384, powers of two)
  int block = 256;          // workgroup size: 128, 256 or 512
  int twc_wave_min = -1;    // TWC: lists longer than this go to a wavefront (< 0: 64)
  int twc_block_min = -1;   // TWC: lists longer than this go to the workgroup (< 0: block)
};

// ---- kernel launchers (defined in the .hip files) -----------------------------

// ingest
hipError_t launch_csr_check(const int32_t* R, const int32_t* C, int64_t V, int64_t E,
                            int64_t* flags_dev, hipStream_t st);
hipError_t launch_row_sort(int32_t* R, int32_t* C, uint32_t* W, int64_t V, const int32_t* rows,
                           int64_t n_rows, uint64_t* scratch, hipStream_t st);
hipError_t launch_find_unsorted(const int32_t* R, const int32_t* C, const uint32_t* W, int64_t V,
                                int32_t* rows_out, uint32_t* count, hipStream_t st);
// Renumber by descending degree (see gr_graph); all outputs preallocated
// (perm, inv [V], R_new [V+1], C_new, W_new [E]).
hipError_t relabel_by_degree(const int32_t* R, const int32_t* C, const uint32_t* W, int64_t V,
                             int64_t E, int32_t* perm, int32_t* inv, int32_t* R_new,
                             int32_t* C_new, uint32_t* W_new, hipStream_t st);
hipError_t launch_unrelabel(const int32_t* R_orig, const int32_t* perm, const int32_t* inv,
                            const int32_t* R_new, const int32_t* C_new, const uint32_t* W_new,
                            int64_t V, int64_t E, int32_t* C, uint32_t* W, hipStream_t st);
hipError_t launch_graph_stats(const int32_t* R, const uint32_t* W, int64_t V, int64_t E,
                              int64_t* out2, hipStream_t st);

// frontier statistics and scan
int stats_grid();
// Degree sum / max / size of the frontier (size read on the device), into slot
// `parity` of the control block; clears the other slot and the two counters.
hipError_t launch_frontier_stats(const int32_t* frontier, const uint32_t* n_f_dev, const int32_t* R,
                                 int64_t* block_sums, Ctrl* ctrl, int parity, uint32_t* zero_a,
                                 uint32_t* zero_b, hipStream_t st);
// The three rotating frontier queues.
struct Queues3 {
  int32_t* q[3];
};
// launch_frontier_stats for the frontier left by a block of device-predicated
// levels that started at queue cur0 (the queue is found on the device from
// the block's level count), so the block needs no read-back of its own.
hipError_t launch_frontier_stats_after_block(const Queues3& qs, int cur0, const int32_t* R,
                                             int64_t* block_sums, Ctrl* ctrl, int parity,
                                             hipStream_t st);
// n_f_dev, when not null, is the frontier size on the device (n_f is then
// ignored), so the kernel can be queued before the host knows the size.
hipError_t launch_frontier_offsets(const int32_t* frontier, int64_t n_f, const int32_t* R,
                                   const int64_t* block_sums, const int64_t* total,
                                   int32_t* offsets, int32_t* rstart, int32_t* chunk_start,
                                   int32_t chunk, hipStream_t st,
                                   const uint32_t* n_f_dev = nullptr);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t st);
// copy *src into host-visible memory, then store seq to *flag (system scope)
// Extra words a publication copies to host memory before its fence (a block
// log, while tracing); n_words = 0: none.
struct PublishExtra {
  const uint32_t* src = nullptr;
  uint32_t* dst = nullptr;
  int n_words = 0;
};
hipError_t launch_publish(const Ctrl* src, Ctrl* host_dst, uint32_t* host_flag, uint32_t seq,
                          hipStream_t st, const PublishExtra& extra = PublishExtra{});
// out[c] = in[inv[c]] for the depth and (nullable) parent arrays (inv: caller
// id -> traversal id)
hipError_t launch_permute_out(const int32_t* inv, int64_t V, const int32_t* depth_in,
                              const int32_t* parent_in, int32_t* depth_out, int32_t* parent_out,
                              hipStream_t st);

// BFS.  Visited state: one array of word pairs, bm[2w + p] = "old" word w
// (depth <= d) and bm[2w + 1 - p] = "live" word w, p = level parity.
hipError_t launch_bfs_init(int32_t* depth, int32_t* parent, int64_t V, uint32_t* bm,
                           int64_t n_words, int32_t source, int32_t* queue, Ctrl* ctrl,
                           hipStream_t st);
// mode: 0 = TWC, 1 = LB_LIGHT (input balanced), 2 = LB (output balanced)
// Parent values are caller ids: perm (nullable) maps renumbered ids back.
hipError_t launch_bfs_push(int mode, bool atomic_parent, const int32_t* frontier,
                           const int32_t* offsets, const int32_t* rstart,
                           const int32_t* chunk_start, int64_t n_f, int64_t m_f, const int32_t* R,
                           const int32_t* C, uint32_t* bm, int p, int32_t* depth, int32_t* parent,
                           const int32_t* perm, int32_t next_depth, int32_t* out_q,
                           uint32_t* out_count, const AdvCfg& cfg, hipStream_t st);
// Push with the non-atomic filter: byte marks (all zero before and after),
// then an ordered compaction of the marked vertices.
hipError_t launch_bfs_push_marks(int mode, const int32_t* frontier, const int32_t* offsets,
                                 const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                 int64_t m_f, const int32_t* R, const int32_t* C, uint32_t* bm,
                                 int p, uint8_t* marks, int32_t* parent, const int32_t* perm,
                                 const AdvCfg& cfg, hipStream_t st);
hipError_t launch_bfs_mark_compact(uint8_t* marks, int64_t V, uint32_t* bm, int p, int32_t* depth,
                                   int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                   hipStream_t st);
// HBM copy of `bytes` (multiple of 16) from src to dst, 16 bytes per lane access.
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
hipError_t launch_bfs_parent_fixup(const int32_t* list, const uint32_t* count, int64_t max_count,
                                   const int32_t* R, const int32_t* C, const uint32_t* bm, int p,
                                   int32_t* parent, const int32_t* perm, hipStream_t st);
// Pull over the bitmap; with rem_q the vertices that stay unvisited with
// neighbours are listed for the next level.
hipError_t launch_bfs_pull(bool lb, int64_t V, const int32_t* R, const int32_t* C, uint32_t* bm,
                           int p, int32_t* depth, int32_t* parent, const int32_t* perm,
                           int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                           int64_t* inspected, int32_t* rem_q, uint32_t* rem_count,
                           hipStream_t st);
// Pull over such a list (*n_list entries, at most max_n), listing the vertices
// that stay unvisited again.
hipError_t launch_bfs_pull_list(const int32_t* list, const uint32_t* n_list, int64_t max_n,
                                const int32_t* R, const int32_t* C, uint32_t* bm, int p,
                                int32_t* depth, int32_t* parent, const int32_t* perm,
                                int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                int64_t* inspected, int32_t* rem_q, uint32_t* rem_count,
                                hipStream_t st);
// Idempotent push (no atomics): survivors of the culling heuristics go to
// cand (at most cap entries are stored; *cand_count may count more).  culls:
// the GR_IDEM_CULL_* bits that are on; log_h: history table size (8, 10, 12).
hipError_t launch_bfs_push_idem(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C,
                                const uint32_t* bm, int p, int32_t* depth, int32_t next_depth,
                                uint32_t culls, int log_h, int32_t* cand, uint32_t* cand_count,
                                int64_t cap, const AdvCfg& cfg, hipStream_t st);
// The exact filter after it: live bits set, each new vertex appended once.
hipError_t launch_bfs_idem_filter(const int32_t* cand, const uint32_t* cand_count, int64_t cap,
                                  int64_t V, uint32_t* bm, int p, const int32_t* depth,
                                  int32_t next_depth, int32_t* out_q, uint32_t* out_count,
                                  hipStream_t st);
// betweenness centrality (levels by counting sort of the depths, then per
// level a push advance with fp64 atomic sums or a pull of the sums; see
// k_bc.hip)
hipError_t launch_bc_levels(const int32_t* depth, const int32_t* R, int64_t V, int32_t source,
                            int32_t n_levels, uint32_t* lvl_n, unsigned long long* lvl_m,
                            double* sigma, double* acc, hipStream_t st);
hipError_t launch_bc_scatter(const int32_t* depth, int64_t V, int32_t n_levels, uint32_t* cursor,
                             int32_t* levels, hipStream_t st);
// push form of either pass over one level (mode 0 = TWC, 2 = LB; the level's
// edges at positions e_base .. of `offsets`)
hipError_t launch_bc_sigma(int mode, const int32_t* frontier, const int32_t* offsets,
                           const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                           int64_t m_f, int64_t e_base, const int32_t* R, const int32_t* C,
                           const int32_t* depth, double* sigma, int32_t next_depth,
                           const AdvCfg& cfg, hipStream_t st);
hipError_t launch_bc_dependency(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, int64_t e_base, const int32_t* R, const int32_t* C,
                                const int32_t* depth, const double* sigma, double* acc,
                                int32_t prev_depth, const AdvCfg& cfg, hipStream_t st);
// per-level chunk maps of both passes for every level at once (offsets:
// the degree scan over all n_r vertices in level order; tab: per level its
// first vertex index, first edge position and first chunk, 3 * n_levels)
hipError_t launch_bc_chunk_map(const int32_t* levels, const int32_t* depth, int64_t n_r,
                               const int32_t* offsets, const int64_t* tab, int32_t n_levels,
                               int32_t chunk, int32_t* chunk_map, hipStream_t st);
// pull form of either pass over one level with the LB mapping of `chunk` edges
// (dependency: acc of the level from its successors at depth `want`;
// otherwise sigma of the level from its predecessors at depth `want`); the
// level's edges sit at positions e_base .. e_base + m_f - 1 of `offsets`
hipError_t launch_bc_pull(bool dependency, const int32_t* frontier, const int32_t* offsets,
                          const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                          int64_t m_f, int64_t e_base, int chunk, const int32_t* C,
                          const int32_t* depth, int32_t want, double* sigma, double* acc,
                          hipStream_t st);
hipError_t launch_bc_finalize(const int32_t* depth, const double* sigma, const double* acc,
                              int64_t V, int32_t source, const int32_t* perm, double* bc,
                              double* sigma_out, hipStream_t st);
// batched SSSP (up to 16 sources per pass; see k_msssp.hip): keys per
// vertex in a row of KS = msssp_row(k) slots; relaxation chunks of
// msssp_chunk(chunk) edges
int msssp_row(int k);
int msssp_chunk(int chunk);
// the near / far split: pairs improved to a distance >= T go to fmask and the
// far pile
struct MsFar {
  uint32_t* fmask;
  int32_t* pile;
  uint32_t* pile_count;
  uint32_t T;
};
// relaxed (nullable, V * KS words): the per-source cull of pairs already
// relaxed with their final distance (cleared by init, raised by relax, read
// and reset by rotate)
hipError_t launch_msssp_init(unsigned long long* keys, int KS, uint32_t* amask, uint32_t* nmask,
                             uint32_t* fmask, uint32_t* relaxed, int64_t V, const int32_t* src_dev,
                             int32_t k, hipStream_t st);
hipError_t launch_msssp_relax(int KS, int chunk, const int32_t* frontier, const int32_t* offsets,
                              const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                              int64_t m_f, const int32_t* C, const uint32_t* W,
                              unsigned long long* keys, const uint32_t* amask, uint32_t* nmask,
                              const MsFar* far, const int32_t* perm, uint32_t* relaxed,
                              int32_t* out_q, uint32_t* out_count, hipStream_t st);
hipError_t launch_msssp_refill(const int32_t* pile, const uint32_t* n_pile, int64_t max_pile,
                               int32_t* pile_next, uint32_t* n_pile_next,
                               const unsigned long long* keys, int KS, uint32_t* fmask,
                               uint32_t* amask, uint32_t T0, uint32_t T1, int32_t* out_q,
                               uint32_t* out_count, hipStream_t st);
// amask of the current frontier cleared; the next frontier's vertices get
// amask = nmask (minus culled pairs), nmask = 0, and those with an active
// source left are appended to out_q (out_count zero before)
hipError_t launch_msssp_rotate(const int32_t* cur_q, const uint32_t* cur_n, int64_t max_cur,
                               const int32_t* next_q, const uint32_t* next_n, int64_t max_next,
                               uint32_t* amask, uint32_t* nmask, const unsigned long long* keys,
                               int KS, uint32_t* relaxed, int32_t* out_q, uint32_t* out_count,
                               hipStream_t st);
hipError_t launch_msssp_finalize(const unsigned long long* keys, int KS, int32_t k,
                                 const int32_t* R, int64_t V, uint32_t* dist, int32_t* pred,
                                 const int32_t* perm, const int32_t* src_orig_dev,
                                 int64_t* reached_edges, hipStream_t st);
// live |= old (live = depth <= d + 1 after level d)
hipError_t launch_bitmap_merge(uint32_t* bm, int p, int64_t n_words, hipStream_t st);

// multi-source BFS (64-bit source masks per vertex); depth / parent are the
// caller's [k][V] arrays in caller ids (perm nullable)
hipError_t launch_ms_seed(const int32_t* src_dev, const int32_t* src_orig_dev, int32_t k,
                          unsigned long long* visit, unsigned long long* front, int32_t* depth,
                          int64_t V, const int32_t* R, Ctrl* ctrl, hipStream_t st);
hipError_t launch_ms_push(int mode, const int32_t* active, const int32_t* offsets,
                          const int32_t* rstart, const int32_t* chunk_start, int64_t n_a,
                          int64_t m_a, const int32_t* R, const int32_t* C,
                          const unsigned long long* front, const unsigned long long* visit,
                          unsigned long long* next, int32_t* touched, uint32_t* n_touched,
                          const AdvCfg& cfg, hipStream_t st);
// pull with parent nullable: when given, the pull writes the parents of the
// vertices it reaches (the finalize of that level then gets parent = nullptr)
hipError_t launch_ms_pull(int64_t V, const int32_t* R, const int32_t* C,
                          const unsigned long long* front, const unsigned long long* visit,
                          unsigned long long full, unsigned long long* next, int32_t* touched,
                          uint32_t* n_touched, int32_t* parent, const int32_t* perm,
                          hipStream_t st);
hipError_t launch_ms_finalize(const int32_t* touched, const uint32_t* n_touched, int64_t max_n,
                              const int32_t* R, const int32_t* C, const unsigned long long* front,
                              unsigned long long* front_next, unsigned long long* visit,
                              unsigned long long* next, int32_t* depth, int32_t* parent,
                              const int32_t* perm, int64_t V, int32_t next_depth, Ctrl* ctrl,
                              hipStream_t st);
hipError_t launch_ms_clear(const int32_t* list, const uint32_t* n, int64_t max_n,
                           unsigned long long* front, hipStream_t st);
struct DlArgs;
// One device-predicated level of the batched BFS (small push levels): the
// expansion as a k_dstep, then finalize and clear, both skipping when a level
// of the block declined (ctrl->dl_stop).  front_cur / front_next alternate by
// level; depth / parent are the pass's output rows.
struct MsLevel {
  const int32_t* R;
  const int32_t* C;
  const unsigned long long* front_cur;
  unsigned long long* front_next;
  unsigned long long* visit;
  unsigned long long* next;
  int32_t* depth;
  int32_t* parent;
  const int32_t* perm;
  int64_t V;
  int32_t next_depth;
};
hipError_t launch_ms_dlevel(const DlArgs& a, const MsLevel& m, int n_blocks, int64_t max_touched,
                            hipStream_t st);
hipError_t launch_ms_teps(const unsigned long long* visit, const int32_t* R, int64_t V, int64_t* out,
                          hipStream_t st);

// selector network
int mlp_tile();
hipError_t launch_mlp_forward(const float* params, const float* X, int32_t n, float* Y,
                              hipStream_t st);
hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T,
                                const float* M, int32_t n, float* partial, float* grad,
                                float* loss, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st);
// Inputs of one selector decision besides the frontier statistics in slot sp
// of the control block: n_u / m_u are the unvisited counts before this
// frontier (0 when not tracked), allowed has bit a set for each allowed action.
struct MlpSelect {
  const float* params;
  int sp;
  int64_t V, E, n_u_before, m_u_before;
  int prev_pull;
  int allowed;
  int after_block;  // n_u / m_u before the frontier: V / E minus the block's visited counts
  // multi-source BFS over ms_k sources: n_u = V - ms_pairs / ms_k and
  // m_u = E - ms_pair_edges / ms_k (the average over the sources of the
  // unvisited counts after the current frontier; 0: not multi-source)
  int ms_k;
};
// The network's predicted log2 step times (pred, +inf where not allowed) and
// its argmin (action) written into the control block, which is then published
// to host memory as launch_publish does; one kernel for both.
hipError_t launch_publish_select(const MlpSelect& m, Ctrl* ctrl, Ctrl* host_dst,
                                 uint32_t* host_flag, uint32_t seq, hipStream_t st,
                                 const PublishExtra& extra = PublishExtra{});

// Device-predicated level blocks (iteration control): up to kDlMaxLevels
// push levels are enqueued back to back; each level kernel first decides on
// the device whether it may run (the previous level ran, the frontier is
// non-empty and within max_n / max_m, and for BFS the direction heuristic
// would still push), so the host reads the control block once per block
// instead of once per level.  Each level appends to q[(cur + 1) % 3] and
// clears the counters of q[(cur + 2) % 3], which nothing reads during it.
constexpr int kDlMaxN = 4096;        // frontier vertices staged in LDS per level
constexpr int kDlMaxLevels = 64;     // levels per block (log capacity)
constexpr uint32_t kDlMaxRefill = 1u << 16;  // SSSP far-pile entries a block may split itself
struct DlArgs {
  const int32_t* R;
  const int32_t* C;
  const int32_t* q_cur;       // frontier of this level
  int32_t* q_next;            // appends
  int32_t cur;                // index of q_cur among the three queues
  int32_t step;               // level index inside the block
  int64_t max_n, max_m;       // run only while n_f <= max_n and m_f <= max_m
  int64_t E;                  // for the push -> pull test
  double do_a;                // push -> pull when m_f > m_u * do_a (< 0: never)
  int64_t V;
  int64_t* log;               // [kDlMaxLevels][3]
  Ctrl* ctrl;
  int32_t edges_vs_all = 0;   // 1: push -> pull when m_f > E * do_a (batched BFS's rule)
};
hipError_t launch_dl_begin(Ctrl* ctrl, int cur, int64_t vm, int64_t vn, uint32_t pq_T,
                           int32_t pq_epoch, int32_t pq_fc, hipStream_t st);
hipError_t launch_bfs_dstep(const DlArgs& a, uint32_t* bm, int p, int32_t* depth, int32_t* parent,
                            const int32_t* perm, int32_t next_depth, int n_blocks, hipStream_t st);
hipError_t launch_sssp_dstep(const DlArgs& a, const uint32_t* W, unsigned long long* keys,
                             int32_t* tags, const int32_t* perm, int32_t next_tag, int n_blocks,
                             hipStream_t st);
// SSSP with the two-level priority queue: improved vertices with dist < T go
// to the next frontier, the others to far pile `fc` (once per epoch).
struct PqState {
  uint32_t T;
  uint32_t delta;
  int32_t epoch;
  int32_t fc;
  int32_t* far_base;          // three piles of V entries
  int32_t* far_tag;
  int64_t V;
  const int32_t* perm;        // predecessor values in caller ids (nullable)
};
hipError_t launch_sssp_pq_relax(int mode, const int32_t* frontier, const int32_t* offsets,
                                const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                int64_t m_f, const int32_t* R, const int32_t* C, const uint32_t* W,
                                unsigned long long* keys, int32_t* tags, int32_t next_tag,
                                const PqState& pq, Ctrl* ctrl, int32_t* out_q, uint32_t* out_count,
                                const AdvCfg& cfg, hipStream_t st);
// Refill: T' = T + delta; far pile fc -> next frontier (T <= dist < T') and
// far pile (fc + 1) % 3 (dist >= T'); entries with dist < T are stale.
hipError_t launch_sssp_pq_refill(const unsigned long long* keys, const PqState& pq, Ctrl* ctrl,
                                 int64_t max_n, int32_t* out_q, uint32_t* out_count, hipStream_t st);
hipError_t launch_sssp_pq_dstep(const DlArgs& a, const uint32_t* W, unsigned long long* keys,
                                int32_t* tags, int32_t next_tag, const PqState& pq, int n_blocks,
                                hipStream_t st);

// The SSSP distance mirror: one byte per vertex, ceil(dist / 2^shift) of an
// earlier moment (255: unknown or too large), an upper bound of the distance
// that screens relaxations before their key gathers.
struct DistMirror {
  uint8_t* p;
  uint32_t shift;
};
// quantum 2^shift for a graph whose largest weight is max_weight: 254 steps
// cover at least four times it
inline uint32_t mirror_shift_for(uint32_t max_weight) {
  uint32_t s = 0;
  while ((254ull << s) < 4ull * max_weight && s < 31) ++s;
  return s;
}
// SSSP
// relaxed (nullable): the cull of vertices already relaxed with their final
// distance (cleared here; raised by the marks relaxation, read by the
// compactions); bin_state (nullable): the distance bins' state, cleared
hipError_t launch_sssp_init(unsigned long long* keys, int32_t* tags, int32_t* far_tag,
                            DistMirror mirror, uint32_t* relaxed, uint32_t* bin_state, int64_t V,
                            Ctrl* ctrl, hipStream_t st);
hipError_t launch_sssp_seed(const int32_t* src_dev, int32_t n, unsigned long long* keys,
                            int32_t* tags, Ctrl* ctrl, hipStream_t st);
// keys hold (dist << 32 | predecessor in caller ids); perm nullable
hipError_t launch_sssp_relax(int mode, const int32_t* frontier, const int32_t* offsets,
                             const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                             int64_t m_f, const int32_t* R, const int32_t* C, const uint32_t* W,
                             unsigned long long* keys, int32_t* tags, const int32_t* perm,
                             int32_t next_tag, int32_t* out_q, uint32_t* out_count, const AdvCfg& cfg,
                             hipStream_t st);
// Relaxation with the non-atomic filter (byte marks, all zero before and after
// the pair of calls), then the ordered list of the marked vertices.  With
// filter, the one-byte distance mirror screens the edges before the key gather;
// the compaction refreshes the mirror of every marked vertex.
hipError_t launch_sssp_relax_marks(int mode, const int32_t* frontier, const int32_t* offsets,
                                   const int32_t* rstart, const int32_t* chunk_start, int64_t n_f,
                                   int64_t m_f, const int32_t* R, const int32_t* C,
                                   const uint32_t* W, unsigned long long* keys,
                                   const int32_t* perm, uint8_t* marks, DistMirror mirror,
                                   uint32_t* relaxed, bool filter, const AdvCfg& cfg,
                                   hipStream_t st);
hipError_t launch_sssp_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                    DistMirror mirror, uint32_t* relaxed, int32_t* out_q,
                                    uint32_t* out_count, hipStream_t st);
// Distance-ordered compaction: the marked vertices (minus the culled ones)
// listed in bins of distance, smallest first; *out_count is set, not added to.
constexpr int kSsspBins = 128;
constexpr int kBinCopies = 8;
constexpr int kSsspBinHist = 0;                                 // [kBinCopies][kSsspBins]
constexpr int kSsspBinCursor = kBinCopies * kSsspBins;          // [kBinCopies][kSsspBins]
constexpr int kSsspBinBase = 2 * kBinCopies * kSsspBins;        // lower bound of the distances
constexpr int kSsspBinWords = 2 * kBinCopies * kSsspBins + 1;
struct SsspBins {
  uint32_t* state;  // kSsspBinWords words
  uint32_t shift;   // bin width 2^shift
};
hipError_t launch_sssp_bin_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                   DistMirror mirror, uint32_t* relaxed, const SsspBins& bins,
                                   int32_t* out_q, uint32_t* out_count, hipStream_t st);
// bin width 2^shift for a graph whose largest weight is max_weight: the bins
// span about two to four times it
inline uint32_t bin_shift_for(uint32_t max_weight) {
  uint32_t span = 1, shift = 0;  // smallest power of two above max_weight
  while (span <= max_weight && span < (1u << 31)) span <<= 1;
  while ((uint64_t)kSsspBins << shift < 2ull * span) ++shift;
  return shift;
}
// Priority-queue form: marked vertices below pq.T go to out_q, the others to
// far pile pq.fc (once per far-pile generation).
hipError_t launch_sssp_pq_mark_compact(uint8_t* marks, int64_t V, const unsigned long long* keys,
                                       DistMirror mirror, uint32_t* relaxed, const PqState& pq,
                                       Ctrl* ctrl, int32_t* out_q, uint32_t* out_count,
                                       hipStream_t st);
// dist / pred written at caller ids; src_orig_dev: the sources in caller ids.
// inv (nullable): caller id -> traversal id of a renumbered graph, and then R
// is the caller's row offsets
hipError_t launch_sssp_finalize(const unsigned long long* keys, const int32_t* R, int64_t V,
                                uint32_t* dist, int32_t* pred, const int32_t* inv,
                                const int32_t* src_orig_dev, int32_t n_src, int64_t* reached_edges,
                                hipStream_t st);

}  // namespace gr
