/*
 * CPU oracle for frontier BFS and SSSP.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this code.  It shares nothing with the GPU library: its own queue,
 * its own heap, its own loops.  It is deliberately plain, single-threaded and
 * slow, so that a reader can check it against the definitions by eye.
 *
 * What it computes (the definitions the traversal method reaches exactly):
 *
 *  BFS (paper Sec. 6.1, breadth-first search; labels and predecessors as in
 *  Alg. 1, Set_Problem_Data):
 *    depth(v)  = fewest edges on a path source -> v, or -1 if none;
 *    parent(v) = min { u : (u,v) in E, depth(u) = depth(v) - 1 } for a reached
 *                v != source; -1 for the source and for unreached vertices.
 *    The paper lets any discoverer write the predecessor; the minimum-id
 *    choice is this implementation's reading that makes the result unique.
 *
 *  SSSP (paper Sec. 3 SSSP example and Sec. 6.2; relaxation of Alg. 1,
 *  Update_Label; non-negative weights permit Dijkstra):
 *    dist(v) = min over paths from any source of the summed uint32 weights
 *              (accumulated in 64 bits), UINT32_MAX if unreachable;
 *    pred(v) = min { u : (u,v) in E, dist(u) + w(u,v) = dist(v) } for v not a
 *              source, -1 otherwise.
 *
 * Both predecessor passes walk every out-edge (u,v) once and keep the minimum
 * qualifying u at v, which is the minimum over in-edges without a transpose.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ERANGE -2
#define OR_ENOMEM -3

/* Breadth-first search with a FIFO queue, then the canonical-parent pass. */
int or_bfs(int64_t n_vertices, const int32_t* row_offsets, const int32_t* col_indices,
           int32_t source, int32_t* depth, int32_t* parent) {
  if (n_vertices < 1 || source < 0 || source >= n_vertices) return OR_EINVAL;
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_vertices);
  if (!queue) return OR_ENOMEM;
  for (int64_t v = 0; v < n_vertices; ++v) {
    depth[v] = -1;
    if (parent) parent[v] = -1;
  }
  int64_t head = 0, tail = 0;
  depth[source] = 0;
  queue[tail++] = source;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int64_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
      int32_t v = col_indices[e];
      if (depth[v] == -1) {
        depth[v] = depth[u] + 1;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  if (parent) {
    for (int64_t u = 0; u < n_vertices; ++u) {
      if (depth[u] < 0) continue;
      for (int64_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
        int32_t v = col_indices[e];
        if (depth[v] == depth[u] + 1 && (parent[v] == -1 || u < parent[v])) parent[v] = (int32_t)u;
      }
    }
  }
  return OR_OK;
}

/* ---- binary min-heap of (distance, vertex), lazy deletion ---------------- */

typedef struct {
  uint64_t dist;
  int32_t v;
} or_item;

static int or_less(or_item a, or_item b) {
  return a.dist < b.dist || (a.dist == b.dist && a.v < b.v);
}

static void or_push(or_item* heap, int64_t* size, or_item x) {
  int64_t i = (*size)++;
  heap[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!or_less(heap[i], heap[p])) break;
    or_item t = heap[i]; heap[i] = heap[p]; heap[p] = t;
    i = p;
  }
}

static or_item or_pop(or_item* heap, int64_t* size) {
  or_item top = heap[0];
  heap[0] = heap[--(*size)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < *size && or_less(heap[l], heap[m])) m = l;
    if (r < *size && or_less(heap[r], heap[m])) m = r;
    if (m == i) break;
    or_item t = heap[i]; heap[i] = heap[m]; heap[m] = t;
    i = m;
  }
  return top;
}

/* Dijkstra from one or more sources (dist = min over sources), then the
 * canonical-predecessor pass.  Returns OR_ERANGE if a finite distance does
 * not fit below UINT32_MAX. */
int or_sssp(int64_t n_vertices, const int32_t* row_offsets, const int32_t* col_indices,
            const uint32_t* weights, const int32_t* sources, int64_t n_sources,
            uint32_t* dist_out, int32_t* pred) {
  if (n_vertices < 1 || n_sources < 1) return OR_EINVAL;
  for (int64_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= n_vertices) return OR_EINVAL;
  int64_t n_edges = row_offsets[n_vertices];
  const uint64_t INF = UINT64_MAX;
  uint64_t* dist = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n_vertices);
  char* done = (char*)calloc((size_t)n_vertices, 1);
  char* is_source = (char*)calloc((size_t)n_vertices, 1);
  or_item* heap = (or_item*)malloc(sizeof(or_item) * (size_t)(n_edges + n_sources + 1));
  if (!dist || !done || !is_source || !heap) {
    free(dist); free(done); free(is_source); free(heap);
    return OR_ENOMEM;
  }
  for (int64_t v = 0; v < n_vertices; ++v) dist[v] = INF;
  int64_t size = 0;
  for (int64_t i = 0; i < n_sources; ++i) {
    int32_t s = sources[i];
    is_source[s] = 1;
    if (dist[s] != 0) {
      dist[s] = 0;
      or_item it = {0, s};
      or_push(heap, &size, it);
    }
  }
  while (size > 0) {
    or_item it = or_pop(heap, &size);
    int32_t u = it.v;
    if (done[u] || it.dist != dist[u]) continue;
    done[u] = 1;
    for (int64_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
      int32_t v = col_indices[e];
      uint64_t cand = dist[u] + (uint64_t)weights[e];
      if (cand < dist[v]) {
        dist[v] = cand;
        or_item nx = {cand, v};
        or_push(heap, &size, nx);
      }
    }
  }
  int rc = OR_OK;
  for (int64_t v = 0; v < n_vertices; ++v) {
    if (dist[v] == INF) dist_out[v] = UINT32_MAX;
    else if (dist[v] >= (uint64_t)UINT32_MAX) { rc = OR_ERANGE; dist_out[v] = UINT32_MAX; }
    else dist_out[v] = (uint32_t)dist[v];
  }
  if (pred) {
    for (int64_t v = 0; v < n_vertices; ++v) pred[v] = -1;
    for (int64_t u = 0; u < n_vertices; ++u) {
      if (dist[u] == INF) continue;
      for (int64_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
        int32_t v = col_indices[e];
        if (is_source[v]) continue;
        if (dist[u] + (uint64_t)weights[e] == dist[v] && (pred[v] == -1 || u < pred[v]))
          pred[v] = (int32_t)u;
      }
    }
  }
  free(dist); free(done); free(is_source); free(heap);
  return rc;
}

/*
 * Betweenness centrality (paper Sec. 6, betweenness centrality: Brandes's
 * formulation, a forward BFS pass that counts shortest paths and a backward
 * pass over the BFS levels that accumulates dependencies).
 *
 * For a source s, with d(v) the hop distance from s:
 *   sigma_s(s) = 1,  sigma_s(w) = sum of sigma_s(v) over edges (v,w) with
 *                    d(w) = d(v) + 1          (number of shortest s-w paths);
 *   delta_s(v) = sum over edges (v,w) with d(w) = d(v) + 1 of
 *                sigma_s(v) / sigma_s(w) * (1 + delta_s(w))
 *                (Brandes' recursion for the dependency of s on v, taken in
 *                decreasing distance, so delta_s(w) is final when used);
 *   bc(v)      = sum over the given sources s != v of delta_s(v).
 * No halving for undirected graphs and no normalisation: bc(v) is the sum of
 * sigma_st(v) / sigma_st over ordered pairs (s, t) with s in the source set,
 * t != s, v not in {s, t}.  All arithmetic in double precision.
 * sigma_last (nullable) receives sigma of the last source (0 where unreached).
 */
int or_bc(int64_t n_vertices, const int32_t* row_offsets, const int32_t* col_indices,
          int64_t n_sources, const int32_t* sources, double* bc, double* sigma_last) {
  if (n_vertices < 1 || n_sources < 1) return OR_EINVAL;
  for (int64_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= n_vertices) return OR_EINVAL;
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_vertices);
  int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_vertices);
  double* sigma = (double*)malloc(sizeof(double) * (size_t)n_vertices);
  double* delta = (double*)malloc(sizeof(double) * (size_t)n_vertices);
  if (!order || !dist || !sigma || !delta) {
    free(order);
    free(dist);
    free(sigma);
    free(delta);
    return OR_ENOMEM;
  }
  for (int64_t v = 0; v < n_vertices; ++v) bc[v] = 0.0;
  for (int64_t i = 0; i < n_sources; ++i) {
    const int32_t s = sources[i];
    for (int64_t v = 0; v < n_vertices; ++v) {
      dist[v] = -1;
      sigma[v] = 0.0;
      delta[v] = 0.0;
    }
    /* forward: FIFO BFS; `order` is the visit order (non-decreasing d) */
    int64_t head = 0, tail = 0;
    dist[s] = 0;
    sigma[s] = 1.0;
    order[tail++] = s;
    while (head < tail) {
      const int32_t v = order[head++];
      for (int64_t e = row_offsets[v]; e < row_offsets[v + 1]; ++e) {
        const int32_t w = col_indices[e];
        if (dist[w] == -1) {
          dist[w] = dist[v] + 1;
          order[tail++] = w;
        }
        if (dist[w] == dist[v] + 1) sigma[w] += sigma[v];
      }
    }
    /* backward: vertices in reverse visit order */
    for (int64_t k = tail - 1; k >= 0; --k) {
      const int32_t v = order[k];
      double acc = 0.0;
      for (int64_t e = row_offsets[v]; e < row_offsets[v + 1]; ++e) {
        const int32_t w = col_indices[e];
        if (dist[w] == dist[v] + 1) acc += sigma[v] / sigma[w] * (1.0 + delta[w]);
      }
      delta[v] = acc;
      if (v != s) bc[v] += acc;
    }
    if (sigma_last && i == n_sources - 1)
      for (int64_t v = 0; v < n_vertices; ++v) sigma_last[v] = sigma[v];
  }
  free(order);
  free(dist);
  free(sigma);
  free(delta);
  return OR_OK;
}
