"""GPU parity of gr_bfs_multi: every row of the k x V outputs equals the
single-source oracle BFS from that row's source (bit-exact depths and
canonical parents), for k spanning several 64-source passes with a ragged
last pass, duplicate sources, and push- and pull-dominated levels."""
import numpy as np
import pytest

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


def check_rows(hg, srcs, d, p):
    d = d.cpu().numpy()
    p = None if p is None else p.cpu().numpy()
    for i, s in enumerate(srcs):
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(s))
        np.testing.assert_array_equal(d[i], ed, err_msg=f"depth row {i} src {s}")
        if p is not None:
            np.testing.assert_array_equal(p[i], ep, err_msg=f"parent row {i} src {s}")


def test_multi_rmat14_two_passes(ctx, rmat14):
    g = gr.Graph.from_host(ctx, rmat14)
    srcs = gg.sources(rmat14, 70, seed=31)
    srcs[5] = srcs[3]  # a duplicate source
    d, p, st = gr.bfs_multi(g, srcs)
    check_rows(rmat14, srcs, d, p)
    exp = sum(oracle.teps_edges(rmat14.row_offsets, oracle.bfs(rmat14.row_offsets,
                                                               rmat14.col_indices, int(s))[0] >= 0)
              for s in srcs)
    assert st["teps_edges"] == exp


def test_multi_grid_and_no_parent(ctx):
    hg = gg.grid(37, 53)
    g = gr.Graph.from_host(ctx, hg)
    srcs = np.array([0, 1, 52, 37 * 53 - 1, 900, 901, 1000], np.int32)
    d, p, _ = gr.bfs_multi(g, srcs)
    check_rows(hg, srcs, d, p)
    d2, p2, _ = gr.bfs_multi(g, srcs, want_parent=False)
    assert p2 is None
    np.testing.assert_array_equal(d2.cpu().numpy(), d.cpu().numpy())


def test_multi_hubs_and_disconnected(ctx):
    # two stars joined by a path, plus an isolated part
    n = 3000
    edges = [(0, i) for i in range(2, 1500)] + [(1, i) for i in range(1500, n)] + [(1499, 1500)]
    edges += [(n, n + 1), (n + 1, n + 2)]
    hg = gg.sort_adjacency(gg.from_edges(n + 4, edges, symmetric=True))
    g = gr.Graph.from_host(ctx, hg)
    srcs = np.array([0, 1, 7, 2999, n, n + 3], np.int32)
    d, p, _ = gr.bfs_multi(g, srcs)
    check_rows(hg, srcs, d, p)


def test_multi_er_policies(ctx):
    hg = gg.erdos_renyi(20000, 12, seed=9)
    g = gr.Graph.from_host(ctx, hg)
    srcs = gg.sources(hg, 64, seed=3)
    # do_a = 0: every level pulls; do_a huge: every level pushes
    for kw in [dict(), dict(lb_light_threshold=0), dict(lb_min_avg_degree=1e9),
               dict(lb_light_threshold=1 << 30), dict(do_a=0.0), dict(do_a=1e9)]:
        d, p, _ = gr.bfs_multi(g, srcs, opts=gr.default_opts(**kw))
        check_rows(hg, srcs, d, p)


def test_multi_errors(ctx, rmat14):
    g = gr.Graph.from_host(ctx, rmat14, symmetric=False)
    with pytest.raises(gr.GrError) as ei:
        gr.bfs_multi(g, [0, 1])
    assert ei.value.code == gr.GR_EUNSUPPORTED
    g2 = gr.Graph.from_host(ctx, rmat14)
    with pytest.raises(gr.GrError) as ei:
        gr.bfs_multi(g2, [0, rmat14.n_vertices])
    assert ei.value.code == gr.GR_EINVAL
