"""Pins of the betweenness-centrality oracle (oracle.bc; paper Sec. 6,
betweenness centrality, Brandes's formulation) against what the mathematics
fixes independently of Brandes' recursion:

  * closed forms (path, star, odd and even cycles, complete graph, complete
    bipartite graph, grid path counts = binomial coefficients);
  * the definition brute-forced on tiny graphs: sigma_st = number of walks of
    length d(s, t) from s to t (every such walk is a shortest path) taken from
    powers of the adjacency matrix, and
    bc(v) = sum over s != v != t with d(s,v) + d(v,t) = d(s,t) of
            sigma_sv * sigma_vt / sigma_st,
    with hop distances from scipy;
  * networkx (its undirected betweenness counts each unordered pair once, so
    the oracle's ordered-pair sum is twice its value).
bc(v) here sums over ordered pairs (s, t) with s in the given sources, with no
halving and no normalisation."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_1701_01170_amd import graphgen as gg


def und(n, edges):
    return gg.from_edges(n, np.array(edges, dtype=np.int64).reshape(-1, 2), None, symmetric=True)


def all_bc(g):
    return oracle.bc(g.row_offsets, g.col_indices, np.arange(g.n_vertices))[0]


@pytest.mark.parametrize("n", [2, 3, 4, 7, 30])
def test_path(n):
    g = und(n, [(i, i + 1) for i in range(n - 1)])
    v = np.arange(n)
    np.testing.assert_array_equal(all_bc(g), 2.0 * v * (n - 1 - v))
    # from the end vertex: every farther target passes through v
    b, sig = oracle.bc(g.row_offsets, g.col_indices, [0], want_sigma=True)
    expect = np.where(v == 0, 0.0, n - 1 - v).astype(np.float64)
    np.testing.assert_array_equal(b, expect)
    np.testing.assert_array_equal(sig, np.ones(n))


@pytest.mark.parametrize("n", [1, 2, 5, 40])
def test_star(n):
    g = und(n + 1, [(0, i) for i in range(1, n + 1)])
    b = all_bc(g)
    assert b[0] == n * (n - 1)
    assert np.all(b[1:] == 0)
    if n >= 2:
        one, _ = oracle.bc(g.row_offsets, g.col_indices, [1])
        assert one[0] == n - 1 and np.all(one[1:] == 0)


@pytest.mark.parametrize("n", [3, 5, 9, 31, 4, 6, 10, 32])
def test_cycle(n):
    g = und(n, [(i, (i + 1) % n) for i in range(n)])
    k = n // 2
    expect = k * (k - 1) if n % 2 else (k - 1) ** 2
    np.testing.assert_allclose(all_bc(g), np.full(n, float(expect)), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 6, 17])
def test_complete_graph(n):
    g = und(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    assert np.all(all_bc(g) == 0)


@pytest.mark.parametrize("m,n", [(1, 3), (2, 2), (3, 5), (4, 7)])
def test_complete_bipartite(m, n):
    # side A = 0..m-1, side B = m..m+n-1: the n(n-1) ordered pairs of B meet at
    # distance 2 through each of the m A vertices with weight 1/m (and vice versa)
    g = und(m + n, [(a, m + b) for a in range(m) for b in range(n)])
    b = all_bc(g)
    np.testing.assert_allclose(b[:m], n * (n - 1) / m, rtol=1e-15)
    np.testing.assert_allclose(b[m:], m * (m - 1) / n, rtol=1e-15)


@pytest.mark.parametrize("rows,cols", [(1, 5), (4, 4), (7, 11)])
def test_grid_path_counts(rows, cols):
    g = gg.grid(rows, cols)
    _, sig = oracle.bc(g.row_offsets, g.col_indices, [0], want_sigma=True)
    r, c = np.divmod(np.arange(rows * cols), cols)
    expect = np.array([math.comb(int(a + b), int(a)) for a, b in zip(r, c)], dtype=np.float64)
    np.testing.assert_array_equal(sig, expect)


def brute_bc(n, R, C, sources):
    """bc from the definition: path counts as walk counts of matrix powers."""
    A = np.zeros((n, n), dtype=object)
    for u in range(n):
        for e in range(R[u], R[u + 1]):
            A[u, C[e]] += 1
    M = sp.csr_matrix((np.ones(len(C)), C, R), shape=(n, n))
    D = shortest_path(M, unweighted=True, directed=True)
    powers = [np.identity(n, dtype=object)]
    for _ in range(n):
        powers.append(powers[-1].dot(A))
    sigma = np.zeros((n, n), dtype=object)
    for s in range(n):
        for t in range(n):
            if np.isfinite(D[s, t]):
                sigma[s, t] = powers[int(D[s, t])][s, t]
    bc = np.zeros(n)
    for s in sources:
        for t in range(n):
            if t == s or not np.isfinite(D[s, t]):
                continue
            for v in range(n):
                if v in (s, t) or not (np.isfinite(D[s, v]) and np.isfinite(D[v, t])):
                    continue
                if D[s, v] + D[v, t] == D[s, t]:
                    bc[v] += float(sigma[s, v] * sigma[v, t]) / float(sigma[s, t])
    return bc, sigma


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("directed", [False, True])
def test_brute_force_tiny(seed, directed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 11))
    m = int(rng.integers(1, 3 * n))
    e = rng.integers(0, n, size=(m, 2))  # self-loops and repeated edges included
    g = gg.from_edges(n, e, None, symmetric=not directed)
    R, C = g.row_offsets, g.col_indices
    srcs = list(range(n)) if seed % 2 == 0 else sorted(rng.choice(n, size=max(1, n // 2), replace=False).tolist())
    expect, sigma = brute_bc(n, R, C, srcs)
    got, sig = oracle.bc(R, C, srcs, want_sigma=True)
    np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12)
    last = srcs[-1]
    np.testing.assert_array_equal(sig, np.array([float(x) for x in sigma[last]]))


def test_networkx_rmat():
    nx = pytest.importorskip("networkx")
    g = gg.rmat(9, 8, seed=3)
    G = nx.Graph()
    G.add_nodes_from(range(g.n_vertices))
    for u in range(g.n_vertices):
        for e in range(g.row_offsets[u], g.row_offsets[u + 1]):
            G.add_edge(u, int(g.col_indices[e]))
    ref = nx.betweenness_centrality(G, normalized=False)
    got = all_bc(g)
    np.testing.assert_allclose(got, 2.0 * np.array([ref[v] for v in range(g.n_vertices)]),
                               rtol=1e-9, atol=1e-9)


def test_networkx_directed():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(5)
    n = 300
    e = np.unique(rng.integers(0, n, size=(1500, 2)), axis=0)
    e = e[e[:, 0] != e[:, 1]]
    g = gg.sort_adjacency(gg.from_edges(n, e, None))
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in e)
    ref = nx.betweenness_centrality(G, normalized=False)
    np.testing.assert_allclose(all_bc(g), np.array([ref[v] for v in range(n)]), rtol=1e-9, atol=1e-9)


def test_source_subset_is_a_sum_over_sources():
    g = gg.rmat(8, 8, seed=4)
    srcs = gg.sources(g, 5, seed=9)
    total, _ = oracle.bc(g.row_offsets, g.col_indices, srcs)
    parts = sum(oracle.bc(g.row_offsets, g.col_indices, [int(s)])[0] for s in srcs)
    np.testing.assert_allclose(total, parts, rtol=1e-12, atol=1e-12)
