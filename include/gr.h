/*
 * gr.h - C ABI of the frontier-centric graph traversal library for AMD
 * Instinct MI355X (gfx950).
 *
 * The library implements the data-centric abstraction of "Gunrock: GPU Graph
 * Analytics" (Wang et al., ACM TOPC 2017): a traversal is a sequence of
 * bulk-synchronous steps that map a vertex frontier to the next one (Sec. 3)
 * using two operators,
 *   - advance: expand the neighbour lists of the frontier (Sec. 4.1, Sec. 5.1:
 *     dynamic grouping "TWC", merge-based load balancing "LB", and pull
 *     traversal over the unvisited vertices, Alg. 2), and
 *   - filter: cull visited vertices, remove duplicates and compact the output
 *     frontier (Sec. 4.2, Sec. 5.2),
 * driving breadth-first search (Sec. 6.1) and single-source shortest paths
 * with atomic-min relaxation (Sec. 6.2, Alg. 1).
 *
 * Conventions for every entry point:
 *   - Return GR_OK (0) or a negative gr_status; gr_last_error() then holds a
 *     message (thread-local, valid until the next failing call on that thread).
 *   - Arguments are validated on the host before any device work is enqueued.
 *     Output contents are unspecified after an error.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; traversal calls return only after their
 *     results are complete (they synchronise the stream).
 *   - Output arrays are caller-owned DEVICE buffers of exactly the stated size.
 *     Index arrays of sources are HOST arrays.
 *   - Graph storage: int32 CSR (row_offsets[V+1], col_indices[E]) with
 *     optional uint32 weights[E] aligned with col_indices (Sec. 5.4).
 *   - Result conventions (Alg. 1, Set_Problem_Data): an unreached vertex has
 *     depth -1, parent -1, distance UINT32_MAX; a source has depth 0 /
 *     distance 0 and parent -1.
 *   - Parents are canonical: among all valid predecessors the one with the
 *     smallest vertex id, so results are unique and do not depend on the
 *     traversal strategy, the schedule or the thread count.
 *   - A gr_ctx and its graphs must not be used by two host threads at once.
 *   - Traversals wait for each step's control block with a wall-clock limit
 *     (60 s, or GR_WAIT_LIMIT_MS from the environment when the context is
 *     created); past it they return GR_EHIP, and the context must then be
 *     destroyed, since its stream may still hold the unfinished work.
 */
#ifndef GR_H
#define GR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GR_ABI_VERSION 6

typedef enum gr_status {
  GR_OK = 0,
  GR_EINVAL = -1,         /* invalid argument or malformed CSR */
  GR_ERANGE = -2,         /* a size or a possible distance exceeds the supported range */
  GR_ENOMEM = -3,         /* device or host allocation failed */
  GR_EHIP = -4,           /* a HIP runtime call failed (message holds the HIP error) */
  GR_ENODEV = -5,         /* no usable gfx950 device */
  GR_EUNSUPPORTED = -6    /* valid request the library cannot serve */
} gr_status;

/* How the per-iteration strategy is chosen (Sec. 5.1 heuristics). */
typedef enum gr_policy {
  GR_POLICY_HEURISTIC = 0, /* the paper's fixed thresholds (average degree, frontier size, do_a/do_b) */
  GR_POLICY_LEARNED = 1,   /* the selector MLP loaded with gr_ctx_set_policy (falls back to heuristic if none) */
  GR_POLICY_FIXED = 2,     /* always opts.fixed_action (pull falls back to push where pull is not allowed) */
  GR_POLICY_RANDOM = 3     /* a seeded random action per iteration (testing: results must not change) */
} gr_policy;

/* Per-iteration advance strategies (Sec. 5.1, Table "traversal strategies"). */
typedef enum gr_action {
  GR_PUSH_TWC = 0, /* push, dynamic grouping by degree: workgroup / wavefront / lane tiers */
  GR_PUSH_LB = 1,  /* push, merge-based load balance (input-balanced below lb_light_threshold) */
  GR_PULL_TWC = 2, /* pull over the unvisited frontier, dynamic grouping per unvisited vertex */
  GR_PULL_LB = 3   /* pull over the unvisited frontier, fixed-width edge groups per vertex */
} gr_action;

/* gr_graph_from_csr flags */
#define GR_SYMMETRIC 0x1u       /* the CSR holds both (u,v) and (v,u) for every edge: pull may use it */
#define GR_DEVICE_INPUT 0x2u    /* row_offsets/col_indices/weights are device pointers */
#define GR_RENUMBER 0x4u        /* renumber vertices by descending degree inside the handle, so the
                                   per-vertex state of hubs shares cache lines (raises the L2 hit
                                   rate of SSSP relaxation on scale-free graphs, but clusters the
                                   long lists of the pull steps); inputs and outputs use the
                                   caller's ids either way and results are identical */

typedef struct gr_ctx gr_ctx;
typedef struct gr_graph gr_graph;

/* One record per iteration when opts.trace is set (features of Sec. 5.1's
 * direction heuristic, plus the measured time of the chosen step). */
typedef struct gr_level_trace {
  int32_t level;       /* iteration index d (frontier = vertices at depth d for BFS) */
  int32_t action;      /* gr_action used */
  int64_t n_f;         /* frontier vertices */
  int64_t m_f;         /* sum of frontier degrees */
  int64_t n_u;         /* unvisited vertices (BFS) */
  int64_t m_u;         /* sum of unvisited degrees (BFS) */
  int64_t max_deg_f;   /* largest frontier degree */
  float features[8];   /* selector input features (see gr_features) */
  float step_us;       /* device time of the whole iteration (advance, filter, bookkeeping) */
  float kernel_us;     /* device time of the advance kernel alone (event-timed) */
  int32_t kernel;      /* advance kernel: 0 TWC, 1 LB_LIGHT, 2 LB, 3 LB with byte-mark filter,
                          4 pull TWC, 5 pull groups (either over the bitmap, or over the
                          short list of still-unvisited vertices the previous pull level
                          left), 6 device-predicated step (step_us and
                          kernel_us are then the block's time divided by its levels),
                          7 SSSP priority-queue refill (far pile split), 8 / 9 / 10 SSSP
                          TWC / LB_LIGHT / LB relaxation with the byte-mark filter,
                          11 BFS pull over the list of still-unvisited vertices the
                          previous pull level left (else 4 / 5 pull over the bitmap),
                          12 / 13 / 14 idempotent BFS push TWC / LB_LIGHT / LB
                          (GR_BFS_FILTER_IDEMPOTENT) */
  int64_t n_next;      /* size of the output frontier */
  int64_t n_in;        /* vertices the advance read as input: push the frontier (n_f),
                          pull over the bitmap the unvisited vertices (n_u), pull over
                          the list its entries, refill the far-pile entries */
  int64_t inspected;   /* edges the advance read: push m_f, pull the neighbours scanned */
  int64_t n_cand;      /* entries the advance emitted before the exact filter: n_next for
                          the exact filters, more with the idempotent advance (its
                          surviving duplicates; see gr_opts.bfs_filter) */
} gr_level_trace;

typedef struct gr_opts {
  uint32_t struct_size;      /* sizeof(gr_opts); set by gr_opts_default */
  int32_t policy;            /* gr_policy */
  int32_t fixed_action;      /* gr_action for GR_POLICY_FIXED */
  int32_t lb_light_threshold;/* PUSH_LB uses input-frontier balance below this frontier size (paper: 4096) */
  uint64_t policy_seed;      /* seed for GR_POLICY_RANDOM */
  float do_a;                /* push -> pull when m_f > m_u * do_a (Sec. 5.1, direction switch) */
  float do_b;                /* pull -> push when m_f < m_u * do_b */
  float lb_min_avg_degree;   /* LB when average degree >= this, else TWC (paper: 5) */
  int32_t max_iterations;    /* stop after this many iterations (<= 0: unlimited) */
  int32_t lb_chunk;          /* edges per workgroup in output-balanced LB: 0 (default 8192), 512, 1024,
                                2048, 4096, 8192, 16384 */
  int32_t trace_capacity;    /* records available in trace */
  gr_level_trace* trace;     /* host array, nullable: per-iteration records */
  int32_t trace_count;       /* out: records written (may exceed capacity; extra are dropped) */
  int32_t device_max_edges;  /* iteration control: while the policy pushes and the frontier has at
                                most 4096 vertices and at most this many edges, levels run in blocks
                                of device-predicated steps with one host round trip per block
                                (heuristic and fixed push policies only).  0: default 262144;
                                < 0: off (one host round trip per level); at most 1 << 24 */
  int32_t sssp_delta;        /* SSSP two-level priority queue (Sec. 5.1, priority queue): improved
                                vertices with dist < T form the next frontier, the rest a far pile;
                                when the frontier empties T grows by sssp_delta and the far pile is
                                split.  0: off (every improved vertex is in the next frontier).
                                Results are identical either way. */
  float learned_margin;      /* GR_POLICY_LEARNED: the network's action replaces the heuristic's only
                                when its predicted log2 step time is lower by more than this
                                (0: plain argmin).  Must be >= 0. */
  int32_t bfs_filter;        /* BFS push levels (outside device-predicated blocks), gr_bfs_filter:
                                how repeated discoveries of a vertex are removed */
  int32_t idem_culls_off;    /* GR_BFS_FILTER_IDEMPOTENT: culling heuristics switched off, a bit
                                set of GR_IDEM_CULL_* (0: all on) */
  int32_t idem_table_log2;   /* GR_BFS_FILTER_IDEMPOTENT: log2 of the entries of the per-workgroup
                                history table: 0 (default 10), 8, 10 or 12 */
  int32_t adv_block;         /* workgroup size of the push advance kernels (TWC, LB_LIGHT, LB):
                                0 (default 256), 128, 256 or 512 */
  int32_t twc_wave_min;      /* TWC tiers (Sec. 5.1 dynamic grouping): neighbour lists longer than
                                this are expanded by one wavefront (0: default 64) ... */
  int32_t twc_block_min;     /* ... and lists longer than this by the whole workgroup (0: default
                                adv_block); must be >= twc_wave_min when both are set */
  int32_t graph_blocks;      /* iteration control: 1 = each block of device-predicated levels (see
                                device_max_edges) is recorded as a hipGraph and launched as one
                                graph (the instantiated graph of a block of the same length is
                                kept in the context and updated); 0 = the block's kernels are
                                enqueued one by one.  Ignored while tracing and by gr_bfs_static. */
  int32_t sssp_opt_off;      /* SSSP refinements of the iterations with the byte-mark filter
                                switched off, a bit set of GR_SSSP_OPT_* (0: all on); none
                                changes the results */
  int32_t sssp_multi_sweep;  /* gr_sssp_multi: 0 = up to 16 sources share each sweep over the
                                graph (one key row per vertex); 1 = one source per sweep, each
                                run as gr_sssp runs it (with its distance-ordered frontier, which
                                a shared sweep cannot give every source).  Same results. */
  int32_t trace_steps_off;   /* with trace: 1 = time only each iteration's advance kernel
                                (kernel_us; step_us left 0), which saves two event records per
                                iteration; 0 = time both (the selector's training data) */
  int32_t bc_dir;            /* gr_bc: how each pass crosses a pair of adjacent levels, a
                                GR_BC_DIR_* for the forward pass | another << 2 for the backward
                                pass.  Push: the level the sums come from sweeps its rows and
                                adds into the other end of each edge with an fp64 atomic; pull:
                                the level the sums belong to sweeps its own rows and gathers
                                them (no atomic per edge).  Auto: per pair, push where the
                                level the sums come from has under a quarter of the other
                                level's edges and under 64 edges per vertex of it, else pull.
                                Same results up to the order of the additions. */
} gr_opts;

/* gr_opts.bc_dir values, per pass */
#define GR_BC_DIR_AUTO 0
#define GR_BC_DIR_PUSH 1
#define GR_BC_DIR_PULL 2

/* gr_opts.sssp_opt_off bits */
#define GR_SSSP_OPT_CULL 1  /* drop from the next frontier a vertex whose edges this iteration
                               already relaxed with its final distance (a further
                               Remove_Redundant, Alg. 1); in gr_sssp_multi per (vertex, source)
                               pair, in every iteration */
#define GR_SSSP_OPT_BINS 2  /* gr_sssp: list the next frontier in bins of distance, smallest
                               first, so that small distances are relaxed first (the ordering aim
                               of the Sec. 5.1 priority queue, without its extra iterations); not
                               used with sssp_delta > 0 nor by gr_sssp_multi */

/* gr_opts.bfs_filter (Sec. 5.2: idempotent vs. non-idempotent operations).
 * Results are identical for all three; only the time differs. */
typedef enum gr_bfs_filter {
  GR_BFS_FILTER_AUTO = 0,       /* atomic bitmap culling on small levels, atomic-free byte marks plus
                                   one ordered compaction on levels with >= V/4 frontier edges */
  GR_BFS_FILTER_ATOMIC = 1,     /* every level: the first atomic OR of a vertex's visited bit
                                   appends it (the exact filter fused into the advance) */
  GR_BFS_FILTER_IDEMPOTENT = 2  /* idempotent advance: no atomics; repeated discoveries are culled
                                   by inexact heuristics (visited bitmap, per-workgroup history
                                   hash table, per-wavefront hash table, depth label) and the
                                   survivors (with the duplicates the heuristics missed) go through
                                   an exact filter pass; symmetric graphs only (elsewhere it acts
                                   as GR_BFS_FILTER_AUTO) */
} gr_bfs_filter;
#define GR_IDEM_CULL_WAVE 0x1u   /* per-wavefront table: one lane per repeated vertex of a batch */
#define GR_IDEM_CULL_HISTORY 0x2u /* per-workgroup history table in LDS */
#define GR_IDEM_CULL_LABEL 0x4u  /* depth label already written this level */

typedef struct gr_run_stats {
  int32_t iterations;        /* bulk-synchronous iterations executed */
  int32_t action_count[4];   /* iterations per gr_action */
  int64_t teps_edges;        /* sum of degrees of reached vertices, summed over sources (Sec. 7 TEPS) */
  int64_t inspected_edges;   /* edges read by advance (push: m_f; pull: neighbours scanned) */
  float device_ms;           /* event-timed device time of the call (after validation/setup) */
  int32_t pad;
} gr_run_stats;

typedef struct gr_graph_info {
  int64_t n_vertices;
  int64_t n_edges;
  int64_t max_degree;
  uint32_t flags;            /* as given to gr_graph_from_csr */
  int32_t weighted;          /* 1 if weights were given */
  uint32_t max_weight;       /* largest weight (0 if unweighted) */
  int32_t resorted;          /* 1 if ingest had to sort some adjacency list */
} gr_graph_info;

/* ---- library, context -------------------------------------------------- */

int32_t gr_abi_version(void);
const char* gr_last_error(void);

/* sizeof() of the ABI structs, for bindings to check their layouts:
 * which = 0 gr_opts, 1 gr_run_stats, 2 gr_level_trace, 3 gr_graph_info;
 * -1 for anything else. */
int32_t gr_abi_sizeof(int32_t which);

/* Fill *opts with defaults: heuristic policy, do_a = 1/14, do_b = 1/576,
 * lb_light_threshold = 4096, lb_min_avg_degree = 5, no trace. */
void gr_opts_default(gr_opts* opts);

/* Create a context on HIP device `device`.  GR_ENODEV if there is no such
 * device or it is not gfx950.  The context owns pooled scratch memory. */
gr_status gr_ctx_create(int32_t device, gr_ctx** out);
gr_status gr_ctx_destroy(gr_ctx* ctx);

/* Load selector MLP parameters (host float array, layout given at
 * gr_mlp_forward): n_params = GR_MLP_N_PARAMS loads one network for every
 * traversal; n_params = 2 * GR_MLP_N_PARAMS loads two, the first for gr_bfs /
 * gr_sssp and the second for gr_bfs_multi.  params = NULL unloads (heuristic
 * again). */
#define GR_MLP_N_PARAMS 1476
gr_status gr_ctx_set_policy(gr_ctx* ctx, const float* params, int32_t n_params);

/* ---- graphs (Sec. 5.4: CSR storage) ----------------------------------- */

/* Host-only validation of a CSR (no device work):
 *   1 <= n_vertices <= 2^31 - 2, 0 <= n_edges <= 2^31 - 1,
 *   row_offsets[0] = 0, row_offsets non-decreasing, row_offsets[V] = n_edges,
 *   0 <= col_indices[i] < n_vertices.  Pointers must be host pointers. */
gr_status gr_validate_csr(int64_t n_vertices, int64_t n_edges, const int32_t* row_offsets,
                          const int32_t* col_indices);

/* Copy a CSR graph into device memory owned by the returned handle.  Inputs
 * are read-only and stay owned by the caller (host pointers unless
 * GR_DEVICE_INPUT; device inputs are validated on the device).  Ingest sorts
 * every adjacency list ascending by neighbour id (weights follow), computes
 * degree statistics and, for SSSP, the largest weight.  weights may be NULL
 * (unweighted: gr_sssp then fails with GR_EINVAL).  Without GR_SYMMETRIC the
 * graph is treated as directed and pull strategies are not used. */
gr_status gr_graph_from_csr(gr_ctx* ctx, int64_t n_vertices, int64_t n_edges,
                            const int32_t* row_offsets, const int32_t* col_indices,
                            const uint32_t* weights, uint32_t flags, void* stream,
                            gr_graph** out);
gr_status gr_graph_free(gr_graph* graph);
gr_status gr_graph_get_info(const gr_graph* graph, gr_graph_info* out);
/* Copy the ingested (sorted) CSR, in the caller's vertex ids, back into
 * caller DEVICE buffers (row_offsets[V+1], col_indices[E], weights[E] or NULL). */
gr_status gr_graph_export(const gr_graph* graph, int32_t* row_offsets, int32_t* col_indices,
                          uint32_t* weights, void* stream);

/* ---- traversals -------------------------------------------------------- */

/* Breadth-first search from `source` (Sec. 6.1; direction-optimising
 * traversal of Alg. 2).  depth: device int32[V] (required); parent: device
 * int32[V] or NULL.  depth(v) = fewest edges from the source; parent(v) = the
 * smallest-id in-neighbour at depth(v) - 1.  opts may be NULL (defaults);
 * stats may be NULL. */
gr_status gr_bfs(gr_ctx* ctx, const gr_graph* graph, int32_t source, int32_t* depth,
                 int32_t* parent, gr_opts* opts, void* stream, gr_run_stats* stats);

/* gr_bfs for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, results and statistics as gr_bfs, but every working array (visited
 * bitmaps, frontier queues, degree scan, unvisited lists, byte marks, control
 * block) is carved from a static device workspace of
 * GR_STATIC_WORKSPACE_BYTES that the library holds on each device it runs on
 * until the process ends; the call makes no hipMalloc / hipFree and no other
 * allocating call.  Its address is looked up when the context is created.
 * The workspace needs about 29.25 * V + E / 128 bytes (plus 8 * V for a
 * GR_RENUMBER graph): a graph that does not fit is rejected with GR_ERANGE
 * before any device work.  The workspace keeps the last call's contents and
 * is shared by every call on the device (all contexts, gr_bfs_static only):
 * calls that overlap on one device race and give undefined results. */
#define GR_STATIC_WORKSPACE_BYTES (64ll << 20)
gr_status gr_bfs_static(gr_ctx* ctx, const gr_graph* graph, int32_t source, int32_t* depth,
                        int32_t* parent, gr_opts* opts, void* stream, gr_run_stats* stats);

/* Shortest paths from n_sources host-given sources (Sec. 6.2, Alg. 1:
 * advance with atomic-min relaxation, filter removing redundant vertices).
 * dist: device uint32[V] (required) = least summed weight from any source;
 * pred: device int32[V] or NULL = smallest-id in-neighbour u with
 * dist(u) + w(u,v) = dist(v) (-1 at sources and unreached vertices).
 * Needs weights.  GR_ERANGE when max_weight * (V - 1) >= 2^32 - 1 (a
 * distance might not fit).  Only push strategies are used. */
gr_status gr_sssp(gr_ctx* ctx, const gr_graph* graph, const int32_t* sources, int32_t n_sources,
                  uint32_t* dist, int32_t* pred, gr_opts* opts, void* stream,
                  gr_run_stats* stats);

/* k independent BFS runs sharing each sweep over the graph (the paper's
 * future-work task parallelism, Sec. 8: several BFS at once).  Sources are
 * processed 64 per pass, one bit per source in per-vertex 64-bit masks.
 * depth: device int32[k][V] (required), parent: device int32[k][V] or NULL,
 * row s holding the single-source result for sources[s].  Needs GR_SYMMETRIC
 * (parents are found by pulling over in-edges).  Per level, the heuristic
 * pulls over every vertex when the vertices active in it carry more than
 * E * opts.do_a edges, else it pushes from them with the opts' LB / TWC knobs;
 * GR_POLICY_FIXED / RANDOM pick the action as for gr_bfs (both pull actions
 * use the one pull kernel), and GR_POLICY_LEARNED runs the selector network
 * (the batched one when two are loaded) in the kernel that publishes each
 * level's statistics, on the features of gr_mlp_forward with n_u / m_u the
 * unvisited vertex and edge counts averaged over the pass's sources and the
 * last feature the pass's number of sources, guarded by learned_margin as for
 * gr_bfs.  Small push levels run in blocks of device-predicated levels as in
 * gr_bfs (device_max_edges; not while tracing or under GR_POLICY_RANDOM).
 * opts.trace records every level. */
gr_status gr_bfs_multi(gr_ctx* ctx, const gr_graph* graph, const int32_t* sources, int32_t k,
                       int32_t* depth, int32_t* parent, gr_opts* opts, void* stream,
                       gr_run_stats* stats);

/* k single-source shortest-path runs sharing each sweep over the graph (the
 * paper's future-work task parallelism, Sec. 8, applied to Alg. 1).  Sources
 * are processed 16 per pass: every vertex keeps one packed (distance,
 * predecessor) key per source of the pass in one row (4, 8 or 16 slots), the
 * frontier is the union of the sources' frontiers with a per-vertex mask of
 * the sources it is active for, and each (frontier edge, active source) pair
 * is relaxed by one lane, the pairs of an edge on neighbouring lanes.  dist:
 * device uint32[k][V] (required), pred: device int32[k][V] or NULL; row s
 * equals gr_sssp with the single source sources[s] (same definitions and
 * canonical predecessors).  Needs weights; GR_ERANGE as gr_sssp.  opts used:
 * lb_chunk (512, 1024 (default here) or 2048 edges per workgroup; other
 * values act as 1024), sssp_delta (> 0: near / far split of the improved
 * (vertex, source) pairs at one threshold for all sources, raised by delta
 * when the frontier runs dry; results unchanged) and max_iterations.  stats:
 * teps_edges summed over the sources; iterations of the longest pass;
 * inspected_edges = frontier edges swept (each once for all its sources). */
gr_status gr_sssp_multi(gr_ctx* ctx, const gr_graph* graph, const int32_t* sources, int32_t k,
                        uint32_t* dist, int32_t* pred, gr_opts* opts, void* stream,
                        gr_run_stats* stats);

/* Betweenness centrality over n_sources host-given sources (Sec. 6,
 * betweenness centrality: Brandes's forward pass counting shortest paths and
 * backward pass accumulating dependencies, both on the advance operator).
 * bc: device double[V] (required) = for every vertex v, the sum over the
 * given sources s != v of delta_s(v) = sum over targets t not in {s, v} of
 * sigma_st(v) / sigma_st, where sigma_st counts shortest s-t paths and
 * sigma_st(v) those through v (no halving for undirected graphs, no
 * normalisation).  sigma: device double[V] or NULL; with exactly one source it
 * receives sigma_sv (the number of shortest paths from the source to v; 0 if
 * unreached, 1 at the source).  Arithmetic in double precision; sums are
 * accumulated with atomic adds in an order that varies, so the last bits may
 * vary from run to run.  Each source runs one gr_bfs with `opts` (its policy
 * and knobs; tracing and max_iterations are ignored), then one advance per
 * pair of adjacent levels in each pass, pushed or pulled as opts->bc_dir says,
 * over LB chunks of lb_chunk edges (TWC for a pushed level where the average
 * degree is below lb_min_avg_degree).  Needs GR_SYMMETRIC (GR_EUNSUPPORTED otherwise).  stats:
 * iterations and teps_edges summed over the sources' BFS runs; device_ms for
 * the whole call. */
gr_status gr_bc(gr_ctx* ctx, const gr_graph* graph, const int32_t* sources, int32_t n_sources,
                double* bc, double* sigma, gr_opts* opts, void* stream, gr_run_stats* stats);

/* ---- selector network (learned per-iteration strategy) -------------------
 *
 * A small MLP predicts, from eight per-iteration features, the log2 step time
 * of each of the four gr_action strategies; GR_POLICY_LEARNED runs the fused
 * inference kernel on the device every iteration and takes the fastest allowed
 * action, guarded by learned_margin.  Where an iteration is small enough for a
 * block of device-predicated push levels (see device_max_edges) the network
 * may turn the heuristic's pull into a push but not a push into a pull, and
 * the levels inside such a block follow the heuristic.  The choice can only
 * change the time taken: every action computes
 * the exact same results.  (The paper picks strategies by fixed thresholds on
 * the degree distribution, Sec. 5.1, and notes in Sec. 7 that the same
 * parameters do not suit every graph; the network replaces the thresholds.)
 *
 * Architecture: 8 -> 32 -> 32 -> 4, ReLU on both hidden layers, fp32.
 * Parameter layout (GR_MLP_N_PARAMS = 1476 floats, row-major):
 *   W1[32][8], b1[32], W2[32][32], b2[32], W3[4][32], b3[4].
 * Features (each log2(1 + x) / 32): n_f, m_f, n_u, m_u, largest frontier
 * degree, V, E, and V if a pull step would first have to build the unvisited
 * frontier (the previous step pushed) else 0 -- the same values as
 * gr_level_trace.features.
 *
 * The training entry points take DEVICE pointers; all work is enqueued on
 * `stream` (asynchronous: they do not synchronise). */

/* Y[n][4] = network(X[n][8]). */
gr_status gr_mlp_forward(gr_ctx* ctx, const float* params, const float* X, int32_t n, float* Y,
                         void* stream);
/* Masked mean squared error L = sum(M * (Y - T)^2) / max(1, sum M) over the
 * batch X[n][8], targets T[n][4], mask M[n][4] (1 = target observed), and its
 * gradient grad[1476] (deterministic summation order).  loss (device float[1])
 * may be NULL. */
gr_status gr_mlp_loss_grad(gr_ctx* ctx, const float* params, const float* X, const float* T,
                           const float* M, int32_t n, float* grad, float* loss, void* stream);
/* One Adam step (Kingma & Ba) on params[1476] with moment buffers m, v and
 * 1-based step count `step`. */
gr_status gr_mlp_adam(gr_ctx* ctx, float* params, const float* grad, float* m, float* v,
                      int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* ---- measurement --------------------------------------------------------- */

/* HBM calibration: copy `bytes` (a positive multiple of 16) between two device
 * buffers the call allocates and frees, `reps` times (after one untimed copy),
 * with a plain kernel that moves 16 bytes per lane access, and report the
 * achieved bandwidth in GB/s counting bytes read plus bytes written.  This is
 * the measured ceiling quoted next to the datasheet HBM peak. */
gr_status gr_copy_bandwidth(gr_ctx* ctx, int64_t bytes, int32_t reps, void* stream, float* gbps);

#ifdef __cplusplus
}
#endif

#endif /* GR_H */
