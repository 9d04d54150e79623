"""Parity at the benchmark's full sizes, with the knobs and launch
configuration bench.py times: R-MAT scale 22 BFS + SSSP (whole outputs
against the oracle) and BC from one source, the 2048 x 2048 grid, 64-source batched BFS on R-MAT
scale 20 (every row's whole output against a single-source oracle run), and the 256-graph disjoint-union SSSP (every
part against a single-source oracle run on that part)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import autotune
from paper_1701_01170_amd import graphgen as gg

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


def _edge_chunks(R, C, chunk=1 << 26):
    """(u, v, e0, e1) for consecutive slices of the edge list, u computed from
    the row offsets of the rows overlapping the slice."""
    E = int(R[-1])
    for e0 in range(0, E, chunk):
        e1 = min(E, e0 + chunk)
        r0 = int(np.searchsorted(R, e0, side="right")) - 1
        r1 = int(np.searchsorted(R, e1, side="left"))
        rows = np.arange(r0, r1, dtype=np.int64)
        starts = np.maximum(R[rows].astype(np.int64), e0)
        ends = np.minimum(R[rows + 1].astype(np.int64), e1)
        u = np.repeat(rows, np.maximum(ends - starts, 0))
        yield u, C[e0:e1].astype(np.int64), e0, e1


def _sample(V, n, seed):
    return np.unique(np.random.default_rng(seed).integers(0, V, n))


def _check_bfs_invariants(R, C, s, depth, parent, n_sample=20_000, chunk=1 << 26):
    """On every edge depth(v) <= depth(u) + 1 when u is reached (so v is
    reached too); the source has depth 0 and no parent; and for a seeded
    sample of vertices (symmetric graph: the in-neighbours are the row) the
    parent is the smallest-id neighbour one level closer, -1 if unreached."""
    for u, v, _, _ in _edge_chunks(R, C, chunk):
        du, dv = depth[u].astype(np.int64), depth[v].astype(np.int64)
        reach_u = du >= 0
        assert (dv[reach_u] >= 0).all()
        assert (dv[reach_u] <= du[reach_u] + 1).all()
    assert depth[s] == 0 and parent[s] == -1
    for v in _sample(len(R) - 1, n_sample, 17):
        if v == s:
            continue
        nb = C[R[v]:R[v + 1]]
        closer = nb[depth[nb] == depth[v] - 1] if depth[v] > 0 else nb[:0]
        expect = int(closer[0]) if len(closer) else -1
        assert parent[v] == expect, (v, parent[v], expect)


def test_rmat22_bfs_sssp_bit_exact(ctx):
    """The headline step exactly as bench.py times it (degree-renumbered
    ingest, its opts constructor, tuned knobs, per-iteration tracing on,
    bench's first timed sources and preallocated outputs), whole outputs
    against the oracle; the traced per-level BFS statistics against the
    oracle's level profile too."""
    import bench
    hg = gg.add_weights(gg.rmat(22, 16, seed=1), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    ob, os_, tb, ts = bench.headline_opts(gr, g)
    V = hg.n_vertices
    out_b = (torch.empty(V, dtype=torch.int32, device="cuda"),
             torch.empty(V, dtype=torch.int32, device="cuda"))
    out_s = (torch.empty(V, dtype=torch.int32, device="cuda"),
             torch.empty(V, dtype=torch.int32, device="cuda"))
    # the first timed source of bench's default run (2 warm-up steps) and of
    # the driver's run (5 warm-up steps); the source list is prefix-stable
    srcs = gg.sources(hg, 10 + 2, seed=1000)
    for s in (int(srcs[2]), int(srcs[5])):
        d, p, sb = gr.bfs(g, s, opts=ob, out=out_b)
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, s)
        np.testing.assert_array_equal(d.cpu().numpy(), ed, err_msg=f"depth src={s}")
        np.testing.assert_array_equal(p.cpu().numpy(), ep, err_msg=f"parent src={s}")
        assert sb["teps_edges"] == oracle.teps_edges(hg.row_offsets, ed >= 0)
        prof = oracle.level_profile(hg.row_offsets, ed)
        assert 0 < ob.trace_count == len(prof) <= ob.trace_capacity
        for t, ref in zip(tb[:ob.trace_count], prof):
            assert (t.level, t.n_f, t.m_f, t.n_u, t.m_u, t.max_deg_f) == (
                ref["level"], ref["n_f"], ref["m_f"], ref["n_u"], ref["m_u"], ref["maxdeg_f"])
        dist, pred, ss = gr.sssp(g, [s], opts=os_, out=out_s)
        edist, epred = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s])
        np.testing.assert_array_equal(dist.cpu().numpy().view(np.uint32), edist,
                                      err_msg=f"dist src={s}")
        np.testing.assert_array_equal(pred.cpu().numpy(), epred, err_msg=f"pred src={s}")
        assert ss["teps_edges"] == oracle.teps_edges(hg.row_offsets, edist != 0xFFFFFFFF)
        assert 0 < os_.trace_count <= os_.trace_capacity
    g.free()


def test_rmat22_bc_tuned(ctx):
    """Betweenness centrality as bench.py times it (R-MAT 22, degree-renumbered
    ingest, the tuner's BC knobs, bench's first BC source): sigma exactly (path
    counts are integers below 2^53 here) and BC within the tolerance of the BC
    parity tests, against the float64 Brandes oracle over the whole graph."""
    hg = gg.rmat(22, 16, seed=1)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    o = autotune.tuned_opts(g, "bc")
    s = int(gg.sources(hg, 4, seed=1300)[0])
    print(f"bc rmat22 source {s} lb_chunk={o.lb_chunk}", flush=True)
    b, sig, st = gr.bc(g, [s], want_sigma=True, opts=o)
    eb, es = oracle.bc(hg.row_offsets, hg.col_indices, [s], want_sigma=True)
    assert es.max() < 2.0 ** 53
    np.testing.assert_array_equal(sig.cpu().numpy(), es)
    got = b.cpu().numpy()
    err = np.abs(got - eb) / np.maximum(1.0, np.abs(eb))
    assert err.max() <= 1e-9, (int(np.argmax(err)), float(err.max()))
    assert st["teps_edges"] == oracle.teps_edges(hg.row_offsets, es > 0)
    g.free()


def test_grid2048_bfs_sssp_bit_exact(ctx):
    hg = gg.add_weights(gg.grid(2048, 2048), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    s = int(gg.sources(hg, 1, seed=1000)[0])
    d, p, _ = gr.bfs(g, s, opts=autotune.tuned_opts(g, "bfs"))
    ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, s)
    np.testing.assert_array_equal(d.cpu().numpy(), ed)
    np.testing.assert_array_equal(p.cpu().numpy(), ep)
    # closed form: hop distance on the grid is the Manhattan distance
    r0, c0 = divmod(s, 2048)
    rr, cc = np.divmod(np.arange(2048 * 2048), 2048)
    assert (ed == np.abs(rr - r0) + np.abs(cc - c0)).all()
    dist, pred, _ = gr.sssp(g, [s], opts=autotune.tuned_opts(g, "sssp"))
    edist, epred = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s])
    np.testing.assert_array_equal(dist.cpu().numpy().view(np.uint32), edist)
    np.testing.assert_array_equal(pred.cpu().numpy(), epred)
    g.free()


def test_rmat20_64_source_batch(ctx):
    """All 64 rows of the batch compared whole with single-source oracle runs:
    generation order with the default knobs, and the bench's configuration
    (degree-renumbered ingest, tuned knobs) under the heuristic and, when a
    trained network is stored, under the learned policy."""
    from paper_1701_01170_amd import selector
    hg = gg.rmat(20, 16, seed=1)
    srcs = gg.sources(hg, 64, seed=2000).astype(np.int32)
    expect = [oracle.bfs(hg.row_offsets, hg.col_indices, int(s)) for s in srcs]
    teps = sum(oracle.teps_edges(hg.row_offsets, ed >= 0) for ed, _ in expect)
    learned = selector.load_policy(ctx)
    try:
        for keep in (False, True):
            g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=keep)
            cfgs = [("default", gr.default_opts())]
            if keep:
                cfgs.append(("tuned", autotune.tuned_opts(g, "bfs_multi")))
                if learned:
                    cfgs.append(("learned", autotune.tuned_opts(g, "bfs_multi",
                                                                policy=gr.POLICY_LEARNED)))
            for name, o in cfgs:
                depth, parent, st = gr.bfs_multi(g, srcs, opts=o)
                depth = depth.cpu().numpy()
                parent = parent.cpu().numpy()
                for i, (ed, ep) in enumerate(expect):
                    msg = f"source {i} renumber={keep} opts={name}"
                    np.testing.assert_array_equal(depth[i], ed, err_msg=msg)
                    np.testing.assert_array_equal(parent[i], ep, err_msg=msg)
                assert st["teps_edges"] == teps
            g.free()
    finally:
        ctx.set_policy(None)


def test_union256_sssp_bit_exact(ctx):
    parts, psrc = gg.small_rmat_batch(256)
    u, voff = gg.disjoint_union(parts)
    g = gr.Graph.from_host(ctx, u, symmetric=True)
    gsrc = (psrc.astype(np.int64) + voff[:-1]).astype(np.int32)
    dist, pred, _ = gr.sssp(g, gsrc, opts=autotune.tuned_opts(g, "sssp"))
    dist = dist.cpu().numpy().view(np.uint32)
    pred = pred.cpu().numpy()
    for i, p in enumerate(parts):
        ed, ep = oracle.sssp(p.row_offsets, p.col_indices, p.weights, [int(psrc[i])])
        a, b = voff[i], voff[i + 1]
        np.testing.assert_array_equal(dist[a:b], ed, err_msg=f"part {i}")
        np.testing.assert_array_equal(pred[a:b], np.where(ep >= 0, ep + a, -1), err_msg=f"part {i}")
    g.free()


def _check_sssp_invariants(R, C, W, s, dist, pred, n_sample=20_000, chunk=1 << 26):
    """On every edge dist(v) <= dist(u) + w(u, v) when u is reached; the
    source has distance 0 and no predecessor; and for a seeded sample of
    vertices (symmetric graph, one weight per undirected edge) the predecessor
    is the smallest-id neighbour u with dist(u) + w = dist(v), -1 if none."""
    INF = np.uint64(0xFFFFFFFF)
    d = dist.astype(np.uint64)
    for u, v, e0, e1 in _edge_chunks(R, C, chunk):
        du, dv = d[u], d[v]
        reach = du != INF
        assert (dv[reach] <= du[reach] + W[e0:e1][reach].astype(np.uint64)).all()
    assert dist[s] == 0 and pred[s] == -1
    for v in _sample(len(R) - 1, n_sample, 19):
        if v == s:
            continue
        nb = C[R[v]:R[v + 1]]
        w = W[R[v]:R[v + 1]].astype(np.uint64)
        tight = nb[(d[nb] != INF) & (d[nb] + w == d[v])] if d[v] != INF else nb[:0]
        expect = int(tight[0]) if len(tight) else -1
        assert pred[v] == expect, (v, pred[v], expect)


def test_rmat25_batched_sampled(ctx):
    """The largest workload (R-MAT scale 25, ~1.05e9 directed edges) with the
    scale-25 run's configuration (degree-renumbered ingest, tuned knobs):
    rows 0, 3, 7, 9 and 15 of the 16-source batched BFS compared whole against
    single-source oracle runs; the 16-source batched SSSP, one of its rows
    checked by the distance and predecessor invariants and another equal to
    the single-source SSSP from its source."""
    hg = gg.add_weights(gg.rmat(25, 16, seed=1), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    srcs = gg.sources(hg, 16, seed=1000).astype(np.int32)
    depth, parent, _ = gr.bfs_multi(g, srcs, opts=autotune.tuned_opts(g, "bfs_multi"))
    for i in (0, 3, 7, 9, 15):
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(srcs[i]))
        np.testing.assert_array_equal(depth[i].cpu().numpy(), ed, err_msg=f"source {i}")
        np.testing.assert_array_equal(parent[i].cpu().numpy(), ep, err_msg=f"source {i}")
    del ed, ep, depth, parent
    dist16, pred16, _ = gr.sssp_multi(g, srcs, opts=autotune.tuned_opts(g, "sssp_multi"))
    d5 = dist16[5].cpu().numpy().view(np.uint32)
    p5 = pred16[5].cpu().numpy()
    d11 = dist16[11].cpu().numpy()
    p11 = pred16[11].cpu().numpy()
    del dist16, pred16
    _check_sssp_invariants(hg.row_offsets, hg.col_indices, hg.weights, int(srcs[5]), d5, p5)
    # row 11 of the batch equals the single-source SSSP from its source
    dist, pred, _ = gr.sssp(g, [int(srcs[11])], opts=autotune.tuned_opts(g, "sssp"))
    np.testing.assert_array_equal(dist.cpu().numpy(), d11)
    np.testing.assert_array_equal(pred.cpu().numpy(), p11)
    g.free()
