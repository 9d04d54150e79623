"""GPU parity of batched shortest paths (gr_sssp_multi: up to 16 sources per
sweep, the paper's Sec. 8 task parallelism applied to Alg. 1) against K
independent single-source runs of the CPU oracle, row by row, bit-exact."""
import numpy as np
import pytest

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu

U32MAX = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


def check(ctx, hg, sources, symmetric=True, renumber=(False, True), opts_list=({},)):
    sources = [int(s) for s in sources]
    exp = [oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s]) for s in sources]
    teps = sum(oracle.teps_edges(hg.row_offsets, d != U32MAX) for d, _ in exp)
    for keep in renumber:
        g = gr.Graph.from_host(ctx, hg, symmetric=symmetric, renumber=keep)
        for kw in opts_list:
            for want_pred in (True, False):
                d, p, st = gr.sssp_multi(g, sources, want_pred=want_pred, opts=gr.default_opts(**kw))
                dn = d.cpu().numpy().view(np.uint32)
                pn = p.cpu().numpy() if want_pred else None
                for i, (ed, ep) in enumerate(exp):
                    msg = f"row {i} src={sources[i]} k={len(sources)} opts={kw} renumber={keep}"
                    np.testing.assert_array_equal(dn[i], ed, err_msg="dist " + msg)
                    if want_pred:
                        np.testing.assert_array_equal(pn[i], ep, err_msg="pred " + msg)
                assert st["teps_edges"] == teps
        g.free()


@pytest.mark.parametrize("k", [1, 3, 5, 16, 37])
def test_rmat14_rows(ctx, rmat14, k):
    srcs = gg.sources(rmat14, k, seed=3000 + k)
    check(ctx, rmat14, srcs)


PQ_OPTS = ({"sssp_delta": 1}, {"sssp_delta": 8}, {"sssp_delta": 40}, {"sssp_delta": 1 << 30})


def test_duplicate_sources_and_chunks(ctx, rmat14):
    s = [int(x) for x in gg.sources(rmat14, 4, seed=3100)]
    srcs = [s[0], s[1], s[0], s[2], s[3], s[1]]
    check(ctx, rmat14, srcs, renumber=(False,),
          opts_list=({}, {"lb_chunk": 512}, {"lb_chunk": 2048}, {"lb_chunk": 16384},
                     {"sssp_opt_off": gr.SSSP_OPT_CULL}, {"sssp_multi_sweep": 1},
                     {"sssp_multi_sweep": 1, "sssp_delta": 8}) + PQ_OPTS)


@pytest.mark.parametrize("k", [4, 16])
def test_priority_queue_rows(ctx, rmat14, k):
    check(ctx, rmat14, gg.sources(rmat14, k, seed=3400 + k), opts_list=PQ_OPTS)


def test_grid_and_er(ctx):
    grid = gg.add_weights(gg.grid(47, 61), seed=7)
    check(ctx, grid, [0, 47 * 61 - 1, 1000, 1500, 2000, 7, 8, 9], renumber=(False,),
          opts_list=({}, {"sssp_delta": 16}))
    er = gg.add_weights(gg.erdos_renyi(20001, 7, seed=5), seed=6, lo=1, hi=3)  # many ties
    check(ctx, er, gg.sources(er, 12, seed=3200))


def test_directed_zero_weights_and_unreached(ctx):
    rng = np.random.default_rng(11)
    V = 6000
    e = rng.integers(0, V, size=(30000, 2))
    w = rng.integers(0, 4, size=30000)  # zero weights included
    hg = gg.sort_adjacency(gg.from_edges(V, e, w))
    check(ctx, hg, [0, 1, 2, 5999, 17, 17, 4000, 3], symmetric=False,
          opts_list=({}, {"sssp_delta": 2}, {"sssp_opt_off": gr.SSSP_OPT_CULL},
                     {"sssp_multi_sweep": 1}))


def test_union_of_small_graphs(ctx):
    parts = [gg.add_weights(gg.rmat(s, 8, seed=20 + s), seed=30 + s) for s in (8, 10, 11, 9)]
    u, voff = gg.disjoint_union(parts)
    check(ctx, u, [int(voff[i]) + 1 for i in range(4)] + [int(voff[1]) + 5], renumber=(False,))


def test_errors(ctx, rmat14):
    g = gr.Graph.from_host(ctx, gg.rmat(8, 4, seed=1), symmetric=True)  # no weights
    with pytest.raises(gr.GrError) as ei:
        gr.sssp_multi(g, [0, 1])
    assert ei.value.code == gr.GR_EINVAL
    g.free()


def test_rmat20_16_sources_all_rows(ctx):
    hg = gg.add_weights(gg.rmat(20, 16, seed=1), seed=101)
    srcs = gg.sources(hg, 16, seed=3300)
    print(f"sssp_multi rmat20 V={hg.n_vertices} E={hg.n_edges} k=16", flush=True)
    # with and without the per-source cull of pairs already relaxed with
    # their final distance (levels of many more chunks than resident
    # workgroups, where pairs do get culled)
    check(ctx, hg, srcs, renumber=(False, True),
          opts_list=({}, {"sssp_delta": 8}, {"sssp_opt_off": gr.SSSP_OPT_CULL},
                     {"sssp_multi_sweep": 1}))
