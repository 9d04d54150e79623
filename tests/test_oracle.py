"""Pins for the CPU oracle: closed forms, hand-worked fixtures, brute force,
library special cases and invariants.  None of these re-type the oracle's own
loops; each is chosen so that a plausible slip in it (a dropped weight, an
off-by-one level, parents taken from out-edges instead of in-edges, max
instead of min) fails at least one test."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from conftest import golden_graph, load_golden
from paper_1701_01170_amd import graphgen as gg

U32MAX = 0xFFFFFFFF


# ---------------------------------------------------------------- helpers --

def brute_force(V, edges):
    """All-pairs hop counts and weighted distances by Floyd-Warshall (pure
    Python, tiny graphs), and canonical predecessors by enumerating every edge."""
    INF = math.inf
    hop = [[INF] * V for _ in range(V)]
    wd = [[INF] * V for _ in range(V)]
    for i in range(V):
        hop[i][i] = 0
        wd[i][i] = 0
    for u, v, w in edges:
        hop[u][v] = min(hop[u][v], 1)
        wd[u][v] = min(wd[u][v], w)
    for k in range(V):
        for i in range(V):
            for j in range(V):
                if hop[i][k] + hop[k][j] < hop[i][j]:
                    hop[i][j] = hop[i][k] + hop[k][j]
                if wd[i][k] + wd[k][j] < wd[i][j]:
                    wd[i][j] = wd[i][k] + wd[k][j]
    return hop, wd


def brute_bfs(V, edges, s):
    hop, _ = brute_force(V, edges)
    depth = [(-1 if hop[s][v] == math.inf else int(hop[s][v])) for v in range(V)]
    parent = [-1] * V
    for v in range(V):
        if v == s or depth[v] < 0:
            continue
        cands = [u for u, x, _ in edges if x == v and depth[u] == depth[v] - 1]
        parent[v] = min(cands)
    return depth, parent


def brute_sssp(V, edges, sources):
    _, wd = brute_force(V, edges)
    dist = [min(wd[s][v] for s in sources) for v in range(V)]
    pred = [-1] * V
    for v in range(V):
        if v in sources or dist[v] == math.inf:
            continue
        cands = [u for u, x, w in edges if x == v and dist[u] + w == dist[v]]
        pred[v] = min(cands)
    dist = [U32MAX if d == math.inf else int(d) for d in dist]
    return dist, pred


def csr_of(V, edges):
    e = np.array([(u, v) for u, v, _ in edges], dtype=np.int64).reshape(-1, 2)
    w = np.array([w for _, _, w in edges], dtype=np.uint32)
    return gg.from_edges(V, e, w)


# ------------------------------------------------------------ golden files --

@pytest.mark.parametrize("name", ["directed7.txt", "undirected_ties8.txt"])
def test_golden_hand_worked(name):
    fx = load_golden(name)
    g = golden_graph(fx)
    for case in fx["bfs"]:
        d, p = oracle.bfs(g.row_offsets, g.col_indices, case["source"])
        np.testing.assert_array_equal(d, case["depth"])
        np.testing.assert_array_equal(p, case["parent"])
    for case in fx["sssp"]:
        d, p = oracle.sssp(g.row_offsets, g.col_indices, g.weights, [case["source"]])
        np.testing.assert_array_equal(d.astype(np.int64), case["dist"])
        np.testing.assert_array_equal(p, case["pred"])


# ------------------------------------------------------------ closed forms --

def path_graph(n):
    return gg.from_edges(n, [(i, i + 1) for i in range(n - 1)], symmetric=True)


def test_path_closed_form():
    n = 50
    g = path_graph(n)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    np.testing.assert_array_equal(d, np.arange(n))
    np.testing.assert_array_equal(p, np.arange(n) - 1)
    # from the far end the roles flip: depth(i) = n-1-i, parent(i) = i+1
    d, p = oracle.bfs(g.row_offsets, g.col_indices, n - 1)
    np.testing.assert_array_equal(d, n - 1 - np.arange(n))
    exp = np.arange(n) + 1
    exp[n - 1] = -1
    np.testing.assert_array_equal(p, exp)


def test_star_closed_form():
    n = 20
    g = gg.from_edges(n + 1, [(0, i) for i in range(1, n + 1)], symmetric=True)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    assert d[0] == 0 and (d[1:] == 1).all()
    assert p[0] == -1 and (p[1:] == 0).all()
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 7)
    assert d[7] == 0 and d[0] == 1 and p[0] == 7 and p[7] == -1
    others = [i for i in range(1, n + 1) if i != 7]
    assert (d[others] == 2).all() and (p[others] == 0).all()


@pytest.mark.parametrize("n", [9, 10])
def test_cycle_closed_form(n):
    g = gg.from_edges(n, [(i, (i + 1) % n) for i in range(n)], symmetric=True)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    i = np.arange(n)
    np.testing.assert_array_equal(d, np.minimum(i, n - i))
    exp = np.where(i < n - i, i - 1, (i + 1) % n)
    exp[(i == n - i)] = i[(i == n - i)] - 1  # antipode of an even cycle: both sides tie -> smaller id
    exp[0] = -1
    np.testing.assert_array_equal(p, exp)


def test_complete_graph_closed_form():
    n = 12
    g = gg.from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], symmetric=True)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 5)
    exp_d = np.ones(n, dtype=np.int32)
    exp_d[5] = 0
    np.testing.assert_array_equal(d, exp_d)
    exp_p = np.full(n, 5)
    exp_p[5] = -1
    np.testing.assert_array_equal(p, exp_p)


def test_binary_tree_closed_form():
    n = 127
    g = gg.from_edges(n, [((i - 1) // 2, i) for i in range(1, n)], symmetric=True)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    i = np.arange(n)
    np.testing.assert_array_equal(d, np.floor(np.log2(i + 1)).astype(int))
    np.testing.assert_array_equal(p[1:], (i[1:] - 1) // 2)


def grid_expected(R, C, r0, c0):
    ids = np.arange(R * C)
    r, c = ids // C, ids % C
    depth = np.abs(r - r0) + np.abs(c - c0)
    parent = np.full(R * C, -1)
    below = r > r0
    parent[below] = ids[below] - C
    above = r < r0
    parent[above & (c > c0)] = ids[above & (c > c0)] - 1
    parent[above & (c < c0)] = ids[above & (c < c0)] + 1
    parent[above & (c == c0)] = ids[above & (c == c0)] + C
    row = r == r0
    parent[row & (c > c0)] = ids[row & (c > c0)] - 1
    parent[row & (c < c0)] = ids[row & (c < c0)] + 1
    return depth, parent


@pytest.mark.parametrize("R,C,r0,c0", [(7, 9, 3, 4), (1, 17, 0, 5), (16, 16, 0, 0), (5, 3, 4, 2)])
def test_grid_manhattan_closed_form(R, C, r0, c0):
    g = gg.grid(R, C)
    src = r0 * C + c0
    d, p = oracle.bfs(g.row_offsets, g.col_indices, src)
    ed, ep = grid_expected(R, C, r0, c0)
    np.testing.assert_array_equal(d, ed)
    np.testing.assert_array_equal(p, ep)
    # constant weights: SSSP distance is weight x Manhattan distance, and the
    # predecessor is the same canonical parent
    W = np.full(g.n_edges, 3, dtype=np.uint32)
    dist, pred = oracle.sssp(g.row_offsets, g.col_indices, W, [src])
    np.testing.assert_array_equal(dist.astype(np.int64), 3 * ed)
    np.testing.assert_array_equal(pred, ep)


def test_disconnected_union():
    a, b = path_graph(5), path_graph(4)
    gg.add_weights(a)
    gg.add_weights(b)
    u, off = gg.disjoint_union([a, b])
    d, p = oracle.bfs(u.row_offsets, u.col_indices, 0)
    assert (d[5:] == -1).all() and (p[5:] == -1).all()
    dist, pred = oracle.sssp(u.row_offsets, u.col_indices, u.weights, [0])
    assert (dist[5:] == U32MAX).all() and (pred[5:] == -1).all()


def test_isolated_source():
    g = gg.from_edges(4, [(1, 2), (2, 3)], symmetric=True)
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    np.testing.assert_array_equal(d, [0, -1, -1, -1])
    np.testing.assert_array_equal(p, [-1, -1, -1, -1])


def test_sssp_overflow_detected():
    g = gg.from_edges(3, [(0, 1), (1, 2)], weights=[0xF0000000, 0x20000000])
    with pytest.raises(OverflowError):
        oracle.sssp(g.row_offsets, g.col_indices, g.weights, [0])


def test_self_loops_and_duplicates():
    # duplicates: the lighter copy decides the distance; self-loops never parent
    g = gg.from_edges(3, [(0, 1), (0, 1), (1, 1), (1, 2), (0, 0)], weights=[9, 2, 1, 5, 1])
    d, p = oracle.bfs(g.row_offsets, g.col_indices, 0)
    np.testing.assert_array_equal(d, [0, 1, 2])
    np.testing.assert_array_equal(p, [-1, 0, 1])
    dist, pred = oracle.sssp(g.row_offsets, g.col_indices, g.weights, [0])
    np.testing.assert_array_equal(dist, [0, 2, 7])
    np.testing.assert_array_equal(pred, [-1, 0, 1])


# ------------------------------------------------------------- brute force --

@st.composite
def small_graphs(draw, directed=None):
    V = draw(st.integers(1, 12))
    m = draw(st.integers(0, 30))
    edges = []
    for _ in range(m):
        u = draw(st.integers(0, V - 1))
        v = draw(st.integers(0, V - 1))
        w = draw(st.integers(0, 9))
        edges.append((u, v, w))
    if directed is None:
        directed = draw(st.booleans())
    if not directed:
        edges = edges + [(v, u, w) for u, v, w in edges]
    n_src = draw(st.integers(1, min(3, V)))
    srcs = sorted(set(draw(st.lists(st.integers(0, V - 1), min_size=n_src, max_size=n_src))))
    return V, edges, srcs


@settings(max_examples=300, deadline=None)
@given(small_graphs())
def test_bfs_brute_force(case):
    V, edges, srcs = case
    g = csr_of(V, edges)
    for s in srcs:
        d, p = oracle.bfs(g.row_offsets, g.col_indices, s)
        bd, bp = brute_bfs(V, edges, s)
        assert d.tolist() == bd
        assert p.tolist() == bp


@settings(max_examples=300, deadline=None)
@given(small_graphs())
def test_sssp_brute_force(case):
    V, edges, srcs = case
    g = csr_of(V, edges)
    d, p = oracle.sssp(g.row_offsets, g.col_indices, g.weights, srcs)
    bd, bp = brute_sssp(V, edges, srcs)
    assert d.tolist() == bd
    assert p.tolist() == bp


# ------------------------------------------------ library special cases --

def test_scipy_and_networkx_cross_check(rmat14):
    import networkx as nx
    import scipy.sparse as sp
    from scipy.sparse.csgraph import dijkstra, shortest_path
    g = rmat14
    V = g.n_vertices
    A = sp.csr_matrix((np.ones(g.n_edges), g.col_indices, g.row_offsets), shape=(V, V))
    Aw = sp.csr_matrix((g.weights.astype(np.float64), g.col_indices, g.row_offsets), shape=(V, V))
    srcs = gg.sources(g, 3, seed=1000)
    hops = shortest_path(A, method="D", unweighted=True, indices=srcs)
    wd = dijkstra(Aw, indices=srcs)
    G = nx.Graph()
    G.add_nodes_from(range(V))
    rows = np.repeat(np.arange(V), g.degrees())
    G.add_edges_from(zip(rows.tolist(), g.col_indices.tolist()))
    for k, s in enumerate(srcs):
        d, _ = oracle.bfs(g.row_offsets, g.col_indices, int(s))
        exp = np.where(np.isinf(hops[k]), -1, hops[k]).astype(np.int64)
        np.testing.assert_array_equal(d, exp)
        nxd = nx.single_source_shortest_path_length(G, int(s))
        exp2 = np.full(V, -1)
        for v, l in nxd.items():
            exp2[v] = l
        np.testing.assert_array_equal(d, exp2)
        dist, _ = oracle.sssp(g.row_offsets, g.col_indices, g.weights, [int(s)])
        expw = np.where(np.isinf(wd[k]), U32MAX, wd[k]).astype(np.int64)
        np.testing.assert_array_equal(dist.astype(np.int64), expw)


def test_unit_weight_sssp_equals_bfs(rmat14):
    # with every weight 1 both definitions coincide: dist = depth, pred = parent
    g = rmat14
    s = int(gg.sources(g, 1, seed=1000)[0])
    d, p = oracle.bfs(g.row_offsets, g.col_indices, s)
    dist, pred = oracle.sssp(g.row_offsets, g.col_indices, np.ones(g.n_edges, np.uint32), [s])
    np.testing.assert_array_equal(np.where(d < 0, U32MAX, d).astype(np.uint32), dist)
    np.testing.assert_array_equal(p, pred)


def test_multi_source_is_min_of_single(rmat14):
    g = rmat14
    srcs = gg.sources(g, 4, seed=77)
    dist, _ = oracle.sssp(g.row_offsets, g.col_indices, g.weights, srcs)
    singles = np.stack([oracle.sssp(g.row_offsets, g.col_indices, g.weights, [int(s)])[0]
                        for s in srcs])
    np.testing.assert_array_equal(dist, singles.min(0))


# -------------------------------------------------------------- invariants --

def check_bfs_invariants(R, C, s, d, p):
    """Every edge (u,v) from a reached u: v reached, depth(v) <= depth(u)+1;
    every reached v != s has an in-neighbour parent one level closer and no
    smaller-id in-neighbour one level closer."""
    R = np.asarray(R, np.int64)
    V = R.shape[0] - 1
    rows = np.repeat(np.arange(V), np.diff(R))
    C = np.asarray(C, np.int64)
    assert d[s] == 0 and p[s] == -1
    reached_u = d[rows] >= 0
    assert (d[C[reached_u]] >= 0).all()
    assert (d[C[reached_u]] <= d[rows[reached_u]] + 1).all()
    rv = (d >= 0) & (np.arange(V) != s)
    assert (p[rv] >= 0).all() and (p[~rv] == -1).all()
    assert (d[p[rv]] == d[rv] - 1).all()
    # minimal: min over in-edges (u,v) with d(u) = d(v)-1 equals p(v)
    good = (d[rows] >= 0) & (d[C] == d[rows] + 1)
    best = np.full(V, np.iinfo(np.int64).max)
    np.minimum.at(best, C[good], rows[good])
    np.testing.assert_array_equal(best[rv], p[rv])


def check_sssp_invariants(R, C, W, srcs, dist, pred):
    R = np.asarray(R, np.int64)
    V = R.shape[0] - 1
    rows = np.repeat(np.arange(V), np.diff(R))
    C = np.asarray(C, np.int64)
    D = dist.astype(np.int64)
    fin = D != U32MAX
    assert (D[srcs] == 0).all()
    e = fin[rows]
    assert (D[C[e]] <= D[rows[e]] + W[e].astype(np.int64)).all()
    src_mask = np.zeros(V, bool)
    src_mask[srcs] = True
    rv = fin & ~src_mask
    assert (pred[rv] >= 0).all() and (pred[~rv] == -1).all()
    tight = e & (D[rows] + W.astype(np.int64) == D[C])
    best = np.full(V, np.iinfo(np.int64).max)
    np.minimum.at(best, C[tight], rows[tight])
    np.testing.assert_array_equal(best[rv], pred[rv])


def test_invariants_rmat14(rmat14):
    g = rmat14
    for s in gg.sources(g, 3, seed=1000):
        d, p = oracle.bfs(g.row_offsets, g.col_indices, int(s))
        check_bfs_invariants(g.row_offsets, g.col_indices, int(s), d, p)
        dist, pred = oracle.sssp(g.row_offsets, g.col_indices, g.weights, [int(s)])
        check_sssp_invariants(g.row_offsets, g.col_indices, g.weights, [int(s)], dist, pred)


PROFILE_KEYS = (("n_f", "level_nf"), ("m_f", "level_mf"), ("maxdeg_f", "level_maxdeg"),
                ("n_u", "level_nu"), ("m_u", "level_mu"))


@pytest.mark.parametrize("name", ["directed7.txt", "undirected_ties8.txt"])
def test_level_profile_golden(name):
    """Per-level n_f, m_f, largest frontier degree, n_u and m_u (the inputs of
    the Sec. 5.1 direction switch and of the selector) against values worked
    out by hand in the fixture; the undirected case keeps two unreachable
    vertices in the unvisited set to the last level."""
    fx = load_golden(name)
    g = golden_graph(fx)
    for case in fx["bfs"]:
        d, _ = oracle.bfs(g.row_offsets, g.col_indices, case["source"])
        prof = oracle.level_profile(g.row_offsets, d)
        assert [x["level"] for x in prof] == list(range(len(case["level_nf"])))
        for key, fkey in PROFILE_KEYS:
            np.testing.assert_array_equal([x[key] for x in prof], case[fkey], err_msg=key)


def test_level_profile_path_closed_form():
    """Path 0-1-...-(n-1) from vertex 0: level d holds vertex d alone (degree
    1 at the ends, 2 inside); the unvisited vertices d+1..n-1 have degree sum
    2 (n - 2 - d) + 1 before the last level and 0 at it."""
    n = 23
    g = path_graph(n)
    d, _ = oracle.bfs(g.row_offsets, g.col_indices, 0)
    prof = oracle.level_profile(g.row_offsets, d)
    assert len(prof) == n
    for x in prof:
        k = x["level"]
        deg = 1 if k in (0, n - 1) else 2
        assert (x["n_f"], x["m_f"], x["maxdeg_f"]) == (1, deg, deg)
        assert x["n_u"] == n - 1 - k
        assert x["m_u"] == (2 * (n - 2 - k) + 1 if k < n - 1 else 0)


def test_level_profile_star_from_leaf_closed_form():
    """Star with centre 0 and leaves 1..n, BFS from leaf 3: level 0 is the
    leaf (degree 1), level 1 the centre (degree n), level 2 the other n - 1
    leaves (degree 1 each); unvisited degree sums 2n - 1, n - 1, 0.  A sum in
    place of the largest degree would give n - 1 at level 2."""
    n = 17
    g = gg.from_edges(n + 1, [(0, i) for i in range(1, n + 1)], symmetric=True)
    d, _ = oracle.bfs(g.row_offsets, g.col_indices, 3)
    prof = oracle.level_profile(g.row_offsets, d)
    got = [(x["n_f"], x["m_f"], x["maxdeg_f"], x["n_u"], x["m_u"]) for x in prof]
    assert got == [(1, 1, 1, n, 2 * n - 1), (1, n, n, n - 1, n - 1), (n - 1, n - 1, 1, 0, 0)]


def test_level_profile_sums(rmat14):
    g = rmat14
    s = int(gg.sources(g, 1, seed=1000)[0])
    d, _ = oracle.bfs(g.row_offsets, g.col_indices, s)
    prof = oracle.level_profile(g.row_offsets, d)
    assert prof[0]["n_f"] == 1 and prof[0]["m_f"] == g.degrees()[s]
    assert sum(x["n_f"] for x in prof) == int((d >= 0).sum())
    assert sum(x["m_f"] for x in prof) == oracle.teps_edges(g.row_offsets, d >= 0)
    for x in prof:
        assert x["n_u"] + sum(y["n_f"] for y in prof if y["level"] <= x["level"]) == g.n_vertices


def test_multi_source_on_disjoint_union_is_per_part():
    """Parts of a block-diagonal union share no edge, so a multi-source run
    with one source per part must reproduce each part's single-source run
    (shifted by the part's vertex offset); this pins the multi-source seeding
    and the source exclusion of the predecessor pass."""
    parts, srcs = gg.small_rmat_batch(6, scale_lo=3, scale_hi=7, seed=5)
    u, voff = gg.disjoint_union(parts)
    gsrc = [int(s + voff[i]) for i, s in enumerate(srcs)]
    dist, pred = oracle.sssp(u.row_offsets, u.col_indices, u.weights, gsrc)
    depth_m = oracle.bfs_multi(u.row_offsets, u.col_indices, gsrc)[0]
    for i, p in enumerate(parts):
        ed, ep = oracle.sssp(p.row_offsets, p.col_indices, p.weights, [int(srcs[i])])
        a, b = voff[i], voff[i + 1]
        assert (dist[a:b] == ed).all()
        assert (pred[a:b] == np.where(ep >= 0, ep + a, -1)).all()
        bd, _ = oracle.bfs(p.row_offsets, p.col_indices, int(srcs[i]))
        # hop counts bound weighted distances from both sides (weights in 1..64)
        reach = bd >= 0
        assert ((ed != U32MAX) == reach).all()
        assert (ed[reach] >= bd[reach]).all() and (ed[reach] <= 64 * bd[reach]).all()
        assert (depth_m[i][a:b] == bd).all()
        assert (depth_m[i][:a] == -1).all() and (depth_m[i][b:] == -1).all()
