"""Batched small-graph SSSP: many independent weighted R-MAT graphs joined
block-diagonally and solved by one multi-source gr_sssp (one source per
part).  The parts share no edge, so each part's distances and predecessors
must equal a single-source run of the oracle on that part alone."""
import numpy as np
import pytest
import torch

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


@pytest.mark.parametrize("n_graphs,lo,hi", [(1, 8, 8), (24, 6, 10), (64, 4, 9)])
def test_union_sssp_matches_per_graph_oracle(ctx, n_graphs, lo, hi):
    parts, srcs = gg.small_rmat_batch(n_graphs, scale_lo=lo, scale_hi=hi, seed=3)
    u, voff = gg.disjoint_union(parts)
    g = gr.Graph.from_host(ctx, u, symmetric=True)
    gsrc = (srcs.astype(np.int64) + voff[:-1]).astype(np.int32)
    for opts in (gr.default_opts(), gr.default_opts(device_max_edges=-1),
                 gr.default_opts(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC),
                 gr.default_opts(sssp_delta=48)):
        dist, pred, st = gr.sssp(g, gsrc, opts=opts)
        dist = dist.cpu().numpy().view(np.uint32)
        pred = pred.cpu().numpy()
        reached = 0
        for i, p in enumerate(parts):
            ed, ep = oracle.sssp(p.row_offsets, p.col_indices, p.weights, [int(srcs[i])])
            a, b = voff[i], voff[i + 1]
            np.testing.assert_array_equal(dist[a:b], ed, err_msg=f"part {i}")
            np.testing.assert_array_equal(pred[a:b], np.where(ep >= 0, ep + a, -1), err_msg=f"part {i}")
            reached += oracle.teps_edges(p.row_offsets, ed != 0xFFFFFFFF)
        assert st["teps_edges"] == reached
    g.free()
