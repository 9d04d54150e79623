"""Parity at the benchmark's full sizes, with the knobs and launch
configuration bench.py times: R-MAT scale 22 BFS + SSSP (whole outputs
against the oracle), the 2048 x 2048 grid, 64-source batched BFS on R-MAT
scale 20 (whole outputs for a sample of the sources, the edge invariants
and tree validity for all), and the 256-graph disjoint-union SSSP (every
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


def _check_bfs_invariants(R, C, s, depth, parent):
    """depth(v) <= depth(u) + 1 on every edge, every reached non-source vertex
    has a parent one level closer that is its smallest-id such neighbour."""
    deg = np.diff(R.astype(np.int64))
    u = np.repeat(np.arange(len(deg)), deg)
    v = C.astype(np.int64)
    du, dv = depth[u].astype(np.int64), depth[v].astype(np.int64)
    reach_u = du >= 0
    assert (dv[reach_u] >= 0).all()
    assert (dv[reach_u] <= du[reach_u] + 1).all()
    assert depth[s] == 0 and parent[s] == -1
    cand = np.where((du >= 0) & (dv == du + 1), u, np.iinfo(np.int64).max)
    best = np.full(len(deg), np.iinfo(np.int64).max)
    np.minimum.at(best, v, cand)
    big = np.iinfo(np.int64).max
    got = np.where(parent >= 0, parent.astype(np.int64), big)
    nonsrc = np.arange(len(deg)) != s
    assert (got[nonsrc] == best[nonsrc]).all()


def test_rmat22_bfs_sssp_bit_exact(ctx):
    hg = gg.add_weights(gg.rmat(22, 16, seed=1), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    ob = autotune.tuned_opts(g, "bfs")
    os_ = autotune.tuned_opts(g, "sssp")
    for s in gg.sources(hg, 2, seed=1000):
        d, p, _ = gr.bfs(g, int(s), opts=ob)
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(s))
        np.testing.assert_array_equal(d.cpu().numpy(), ed)
        np.testing.assert_array_equal(p.cpu().numpy(), ep)
        dist, pred, _ = gr.sssp(g, [int(s)], opts=os_)
        edist, epred = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [int(s)])
        np.testing.assert_array_equal(dist.cpu().numpy().view(np.uint32), edist)
        np.testing.assert_array_equal(pred.cpu().numpy(), epred)
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
    hg = gg.rmat(20, 16, seed=1)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    srcs = gg.sources(hg, 64, seed=2000).astype(np.int32)
    depth, parent, st = gr.bfs_multi(g, srcs)
    depth = depth.cpu().numpy()
    parent = parent.cpu().numpy()
    teps = 0
    for i, s in enumerate(srcs):
        if i % 16 == 0:
            ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(s))
            np.testing.assert_array_equal(depth[i], ed, err_msg=f"source {i}")
            np.testing.assert_array_equal(parent[i], ep, err_msg=f"source {i}")
        else:
            _check_bfs_invariants(hg.row_offsets, hg.col_indices, int(s), depth[i], parent[i])
        teps += oracle.teps_edges(hg.row_offsets, depth[i] >= 0)
    assert st["teps_edges"] == teps
    g.free()


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
