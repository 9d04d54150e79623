/*
 * Seeded synthetic graph generators (host C, OpenMP).
 *
 * This module produces the inputs that both the GPU traversal library and the
 * CPU oracle consume.  It holds none of the traversal arithmetic: it only draws
 * graphs, weights and sources, deterministically from a seed.
 *
 * Workload definitions follow the paper's evaluation setup (Sec. 7, dataset
 * paragraph): R-MAT graphs with edge factor 16 and initiator a=0.57, b=0.19,
 * c=0.19, d=0.05 (the Graph 500 setting), undirected, with self-loops and
 * duplicate edges removed, and edge weights drawn uniformly from 1..64.
 *
 * Readings where the paper is silent:
 *  - R-MAT: no noise; edge factor k means k * 2^scale generated undirected
 *    pairs; optional seeded vertex relabelling (Graph 500 convention).
 *  - Weights of an undirected edge {u,v} are one value for both directions:
 *    w = lo + H(seed, min(u,v), max(u,v)) mod (hi - lo + 1).
 *
 * Randomness is counter based (a splitmix64-style finaliser applied to
 * (seed, stream, counter)), so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct gg_csr {
  int64_t n_vertices;
  int64_t n_edges;
  int32_t* row_offsets; /* [n_vertices + 1] */
  int32_t* col_indices; /* [n_edges] */
} gg_csr;

/* ---- counter-based random numbers ---------------------------------------- */

static inline uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* One 64-bit draw for (seed, stream, counter). */
static inline uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t k = gg_mix64(seed + 0x9e3779b97f4a7c15ULL * (stream + 1));
  return gg_mix64(k + 0x9e3779b97f4a7c15ULL * (ctr + 1));
}

uint64_t gg_hash3(uint64_t seed, uint64_t a, uint64_t b) {
  return gg_mix64(gg_draw(seed, a, b) ^ 0x5851f42d4c957f2dULL);
}

/* ---- parallel LSD radix sort of 64-bit keys ------------------------------ */

static void gg_radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t n) {
  if (n <= 1) return;
  int nthreads = omp_get_max_threads();
  int64_t* hist = (int64_t*)malloc(sizeof(int64_t) * 256 * (size_t)nthreads);
  uint64_t* src = keys;
  uint64_t* dst = tmp;
  for (int byte = 0; byte < 8; ++byte) {
    int shift = byte * 8;
    memset(hist, 0, sizeof(int64_t) * 256 * (size_t)nthreads);
#pragma omp parallel num_threads(nthreads)
    {
      int t = omp_get_thread_num();
      int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
      int64_t* h = hist + 256 * t;
      for (int64_t i = lo; i < hi; ++i) h[(src[i] >> shift) & 255]++;
    }
    /* skip a pass where every key has the same digit */
    int64_t total_bucket0 = 0;
    int single = 0;
    for (int d = 0; d < 256; ++d) {
      int64_t s = 0;
      for (int t = 0; t < nthreads; ++t) s += hist[256 * t + d];
      if (s == n) single = 1;
      (void)total_bucket0;
    }
    if (single) continue;
    int64_t run = 0;
    for (int d = 0; d < 256; ++d)
      for (int t = 0; t < nthreads; ++t) {
        int64_t c = hist[256 * t + d];
        hist[256 * t + d] = run;
        run += c;
      }
#pragma omp parallel num_threads(nthreads)
    {
      int t = omp_get_thread_num();
      int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
      int64_t* h = hist + 256 * t;
      for (int64_t i = lo; i < hi; ++i) {
        uint64_t k = src[i];
        dst[h[(k >> shift) & 255]++] = k;
      }
    }
    uint64_t* sw = src; src = dst; dst = sw;
  }
  if (src != keys) memcpy(keys, src, sizeof(uint64_t) * (size_t)n);
  free(hist);
}

/* Symmetrise, drop self-loops, sort, deduplicate and build an int32 CSR from a
 * list of undirected pairs packed as (u << 32 | v).  Consumes `pairs`. */
static int gg_pairs_to_csr(uint64_t* pairs, int64_t n_pairs, int64_t n_vertices, gg_csr* out) {
  int64_t cap = 2 * n_pairs;
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1));
  if (!keys) return -3;
  /* count non-loop pairs per thread to place both directions compactly */
  int nthreads = omp_get_max_threads();
  int64_t* cnt = (int64_t*)calloc((size_t)nthreads + 1, sizeof(int64_t));
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int64_t lo = n_pairs * t / nthreads, hi = n_pairs * (t + 1) / nthreads, c = 0;
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t p = pairs[i];
      if ((p >> 32) != (p & 0xffffffffULL)) ++c;
    }
    cnt[t + 1] = c;
  }
  for (int t = 0; t < nthreads; ++t) cnt[t + 1] += cnt[t];
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int64_t lo = n_pairs * t / nthreads, hi = n_pairs * (t + 1) / nthreads;
    int64_t w = 2 * cnt[t];
    for (int64_t i = lo; i < hi; ++i) {
      uint64_t p = pairs[i];
      uint64_t u = p >> 32, v = p & 0xffffffffULL;
      if (u == v) continue;
      keys[w++] = (u << 32) | v;
      keys[w++] = (v << 32) | u;
    }
  }
  int64_t n_keys = 2 * cnt[nthreads];
  free(cnt);
  free(pairs);
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n_keys > 0 ? n_keys : 1));
  if (!tmp) { free(keys); return -3; }
  gg_radix_sort_u64(keys, tmp, n_keys);
  free(tmp);
  int64_t m = 0;
  for (int64_t i = 0; i < n_keys; ++i)
    if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
  if (m > INT32_MAX) { free(keys); return -2; }
  int32_t* R = (int32_t*)calloc((size_t)n_vertices + 1, sizeof(int32_t));
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!R || !C) { free(keys); free(R); free(C); return -3; }
  for (int64_t i = 0; i < m; ++i) R[(keys[i] >> 32) + 1]++;
  for (int64_t v = 0; v < n_vertices; ++v) R[v + 1] += R[v];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) C[i] = (int32_t)(keys[i] & 0xffffffffULL);
  free(keys);
  out->n_vertices = n_vertices;
  out->n_edges = m;
  out->row_offsets = R;
  out->col_indices = C;
  return 0;
}

/* Seeded uniform permutation of [0, n) (Fisher-Yates driven by counter draws). */
static int32_t* gg_permutation(int64_t n, uint64_t seed) {
  int32_t* p = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!p) return NULL;
  for (int64_t i = 0; i < n; ++i) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t r = gg_draw(seed, 7, (uint64_t)i);
    int64_t j = (int64_t)(((unsigned __int128)r * (unsigned __int128)(i + 1)) >> 64);
    int32_t t = p[i]; p[i] = p[j]; p[j] = t;
  }
  return p;
}

/* R-MAT graph: n_pairs = edge_factor * 2^scale undirected pairs, each drawn by
 * `scale` recursive quadrant choices with probabilities (a, b, c, 1-a-b-c). */
int gg_rmat(int scale, double edge_factor, double a, double b, double c,
            uint64_t seed, int permute, gg_csr* out) {
  if (scale < 1 || scale > 30 || edge_factor <= 0 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
    return -1;
  int64_t n = (int64_t)1 << scale;
  int64_t n_pairs = (int64_t)(edge_factor * (double)n + 0.5);
  const double two32 = 4294967296.0;
  uint64_t ta = (uint64_t)(a * two32), tb = (uint64_t)((a + b) * two32), tc = (uint64_t)((a + b + c) * two32);
  uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n_pairs > 0 ? n_pairs : 1));
  if (!pairs) return -3;
  int32_t* perm = permute ? gg_permutation(n, seed ^ 0x7065726dULL) : NULL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_pairs; ++i) {
    uint64_t u = 0, v = 0, h = 0;
    for (int l = 0; l < scale; ++l) {
      uint64_t r;
      if ((l & 1) == 0) { h = gg_draw(seed, 1, (uint64_t)i * 16 + (uint64_t)(l >> 1)); r = h >> 32; }
      else r = h & 0xffffffffULL;
      uint64_t bu, bv;
      if (r < ta) { bu = 0; bv = 0; }
      else if (r < tb) { bu = 0; bv = 1; }
      else if (r < tc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (perm) { u = (uint64_t)perm[u]; v = (uint64_t)perm[v]; }
    pairs[i] = (u << 32) | v;
  }
  free(perm);
  return gg_pairs_to_csr(pairs, n_pairs, n, out);
}

/* Erdos-Renyi style graph: n * avg_degree / 2 uniform undirected pairs. */
int gg_erdos_renyi(int64_t n, double avg_degree, uint64_t seed, gg_csr* out) {
  if (n < 1 || n > INT32_MAX - 1 || avg_degree < 0) return -1;
  int64_t n_pairs = (int64_t)((double)n * avg_degree / 2.0 + 0.5);
  uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n_pairs > 0 ? n_pairs : 1));
  if (!pairs) return -3;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_pairs; ++i) {
    uint64_t h = gg_draw(seed, 2, (uint64_t)i);
    uint64_t u = (uint64_t)(((unsigned __int128)(h >> 32) * (unsigned __int128)n) >> 32);
    uint64_t v = (uint64_t)(((unsigned __int128)(h & 0xffffffffULL) * (unsigned __int128)n) >> 32);
    pairs[i] = (u << 32) | v;
  }
  return gg_pairs_to_csr(pairs, n_pairs, n, out);
}

/* rows x cols 4-neighbour grid, no wrap, row-major ids, ascending adjacency. */
int gg_grid(int64_t rows, int64_t cols, gg_csr* out) {
  if (rows < 1 || cols < 1 || rows * cols > INT32_MAX - 1) return -1;
  int64_t n = rows * cols;
  int64_t m = 2 * (rows * (cols - 1) + cols * (rows - 1));
  int32_t* R = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* C = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!R || !C) { free(R); free(C); return -3; }
  R[0] = 0;
  for (int64_t id = 0; id < n; ++id) {
    int64_t r = id / cols, c = id % cols;
    R[id + 1] = R[id] + (r > 0) + (c > 0) + (c + 1 < cols) + (r + 1 < rows);
  }
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < n; ++id) {
    int64_t r = id / cols, c = id % cols, w = R[id];
    if (r > 0) C[w++] = (int32_t)(id - cols);
    if (c > 0) C[w++] = (int32_t)(id - 1);
    if (c + 1 < cols) C[w++] = (int32_t)(id + 1);
    if (r + 1 < rows) C[w++] = (int32_t)(id + cols);
  }
  out->n_vertices = n;
  out->n_edges = m;
  out->row_offsets = R;
  out->col_indices = C;
  return 0;
}

void gg_free(gg_csr* g) {
  if (!g) return;
  free(g->row_offsets);
  free(g->col_indices);
  g->row_offsets = NULL;
  g->col_indices = NULL;
}

/* Copy a generated CSR into caller buffers and release it. */
void gg_take(gg_csr* g, int32_t* row_offsets, int32_t* col_indices) {
  memcpy(row_offsets, g->row_offsets, sizeof(int32_t) * (size_t)(g->n_vertices + 1));
  if (g->n_edges > 0) memcpy(col_indices, g->col_indices, sizeof(int32_t) * (size_t)g->n_edges);
  gg_free(g);
}

/* Symmetric edge weights: w(u,v) = w(v,u) = lo + H(seed, min, max) mod (hi-lo+1). */
void gg_weights(int64_t n_vertices, const int32_t* row_offsets, const int32_t* col_indices,
                uint64_t seed, uint32_t lo, uint32_t hi, uint32_t* weights) {
  uint64_t span = (uint64_t)hi - (uint64_t)lo + 1;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n_vertices; ++u) {
    for (int64_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
      uint64_t v = (uint64_t)col_indices[e];
      uint64_t a = (uint64_t)u < v ? (uint64_t)u : v, b = (uint64_t)u < v ? v : (uint64_t)u;
      weights[e] = lo + (uint32_t)(gg_hash3(seed, a, b) % span);
    }
  }
}

/* k seeded sources, uniform over vertices with degree > 0 (with replacement
 * across the k draws; draw i uses counters (i, attempt)).  Returns the number
 * of sources written (0 when the graph has no edges). */
int64_t gg_sources(int64_t n_vertices, const int32_t* row_offsets, uint64_t seed, int64_t k,
                   int32_t* out) {
  int64_t nonisolated = 0;
  for (int64_t v = 0; v < n_vertices; ++v) nonisolated += row_offsets[v + 1] > row_offsets[v];
  if (nonisolated == 0) return 0;
  for (int64_t i = 0; i < k; ++i) {
    for (uint64_t attempt = 0;; ++attempt) {
      uint64_t r = gg_draw(seed, 3, (uint64_t)i * 1000003ULL + attempt);
      int64_t v = (int64_t)(((unsigned __int128)r * (unsigned __int128)n_vertices) >> 64);
      if (row_offsets[v + 1] > row_offsets[v]) { out[i] = (int32_t)v; break; }
    }
  }
  return k;
}
