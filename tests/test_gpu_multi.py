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


MULTI_POLICIES = [
    ("fixed_push_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC)),
    ("fixed_push_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB)),
    ("fixed_pull", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_TWC)),
    ("fixed_pull_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_LB)),
    ("random7", dict(policy=gr.POLICY_RANDOM, policy_seed=7)),
    ("random8", dict(policy=gr.POLICY_RANDOM, policy_seed=8, lb_light_threshold=0)),
    ("learned", dict(policy=gr.POLICY_LEARNED)),
    ("learned_margin", dict(policy=gr.POLICY_LEARNED, learned_margin=0.25)),
]


def test_multi_policies_change_only_time(ctx, rmat14):
    """Every per-level action choice of the batched BFS gives the oracle's
    rows: fixed, random and learned policies (the learned one with a random
    network for the batched traversal, so its choices vary)."""
    rng = np.random.default_rng(4)
    single = rng.standard_normal(gr.MLP_N_PARAMS).astype(np.float32)
    multi = rng.standard_normal(gr.MLP_N_PARAMS).astype(np.float32)
    for hg in (rmat14, gg.grid(41, 29)):
        g = gr.Graph.from_host(ctx, hg)
        srcs = gg.sources(hg, 40, seed=77)
        for loaded in (None, np.concatenate([single, multi]), single):
            ctx.set_policy(loaded)
            for name, kw in MULTI_POLICIES:
                d, p, st = gr.bfs_multi(g, srcs, opts=gr.default_opts(**kw))
                check_rows(hg, srcs, d, p)
        ctx.set_policy(None)
        g.free()


def test_multi_trace_records(ctx, rmat14):
    """The batched BFS traces every level: its frontier statistics, the action
    taken, and the unvisited counts averaged over the sources."""
    g = gr.Graph.from_host(ctx, rmat14)
    srcs = gg.sources(rmat14, 16, seed=78)
    cap = 256
    tr = (gr.LevelTrace * cap)()
    o = gr.default_opts(trace=tr, trace_capacity=cap, policy=gr.POLICY_RANDOM, policy_seed=3)
    d, p, st = gr.bfs_multi(g, srcs, opts=o)
    check_rows(rmat14, srcs, d, p)
    recs = tr[:o.trace_count]
    assert len(recs) == st["iterations"] > 0
    dn = d.cpu().numpy()
    R = rmat14.row_offsets
    deg = np.diff(R).astype(np.int64)
    for r in recs:
        active = (dn == r.level).any(axis=0)
        assert r.n_f == int(active.sum())
        assert r.m_f == int(deg[active].sum())
        reached = (dn >= 0) & (dn <= r.level)
        assert r.n_u == rmat14.n_vertices - int(reached.sum()) // len(srcs)
        assert r.m_u == rmat14.n_edges - int((reached * deg[None, :]).sum()) // len(srcs)
        assert r.step_us > 0
    assert [r.action for r in recs].count(gr.PULL_TWC) + [r.action for r in recs].count(gr.PULL_LB) \
        == st["action_count"][2] + st["action_count"][3]


@pytest.mark.parametrize("kw", [dict(device_max_edges=-1), dict(device_max_edges=64),
                                dict(device_max_edges=1 << 24),
                                dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB,
                                     device_max_edges=1 << 24)])
def test_multi_device_blocks(ctx, kw):
    """Small push levels of the batched BFS run in device-predicated blocks
    (finalize and clear predicated on the block's stop flag): off, stopped by a
    tiny edge bound, covering every push level, and under a fixed push policy."""
    for hg in (gg.grid(61, 47), gg.rmat(13, 8, seed=5)):
        g = gr.Graph.from_host(ctx, hg)
        srcs = gg.sources(hg, 37, seed=91)
        d, p, st = gr.bfs_multi(g, srcs, opts=gr.default_opts(**kw))
        check_rows(hg, srcs, d, p)
        g.free()


@pytest.mark.parametrize("cap", [1, 2, 5, 9, 40])
def test_multi_max_iterations(ctx, cap):
    """A level cap (also one that falls inside a device block) keeps exactly
    the levels it allows: depths up to the cap, their parents."""
    hg = gg.grid(33, 29)
    g = gr.Graph.from_host(ctx, hg)
    srcs = np.array([0, 500, 956], np.int32)
    d, p, st = gr.bfs_multi(g, srcs, opts=gr.default_opts(max_iterations=cap))
    dn, pn = d.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(srcs):
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(s))
        keep = (ed >= 0) & (ed <= cap)
        np.testing.assert_array_equal(dn[i], np.where(keep, ed, -1), err_msg=f"row {i}")
        np.testing.assert_array_equal(pn[i], np.where(keep, ep, -1), err_msg=f"row {i}")
    assert st["iterations"] == min(cap, max(int(oracle.bfs(hg.row_offsets, hg.col_indices, int(s))[0].max())
                                             for s in srcs) + 1)
    g.free()


def test_batched_network_gain_on_grid(ctx):
    """What the trained batched-BFS network gains over the method without it:
    64 sources on a 384 x 384 grid (a held-out graph of the network's
    evaluation), where the heuristic's push -> pull switch pulls about half of
    the levels and the network keeps pushing, which is faster on this
    small-frontier, high-diameter graph.  Both policies give the same rows; the
    learned run is faster (best of three each, interleaved)."""
    from paper_1701_01170_amd import autotune, selector
    if not selector.load_policy(ctx):
        pytest.skip("no trained network stored")
    try:
        hg = gg.grid(384, 384)
        g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
        srcs = gg.sources(hg, 64, seed=9100).astype(np.int32)
        cfgs = {"heuristic": autotune.tuned_opts(g, "bfs_multi"),
                "learned": autotune.tuned_opts(g, "bfs_multi", policy=gr.POLICY_LEARNED)}
        best = {k: float("inf") for k in cfgs}
        rows, actions = {}, {}
        for _ in range(3):
            for label, o in cfgs.items():
                d, p, st = gr.bfs_multi(g, srcs, opts=o)
                best[label] = min(best[label], st["device_ms"])
                rows[label] = (d.cpu().numpy(), p.cpu().numpy())
                actions[label] = st["action_count"]
        np.testing.assert_array_equal(rows["learned"][0], rows["heuristic"][0])
        np.testing.assert_array_equal(rows["learned"][1], rows["heuristic"][1])
        check_rows(hg, srcs[:2], *(torch_rows(rows["learned"], 2)))
        print(f"grid 384 x 384, 64 sources: heuristic {best['heuristic']:.3f} ms "
              f"(actions {actions['heuristic']}), learned {best['learned']:.3f} ms "
              f"(actions {actions['learned']})", flush=True)
        assert best["learned"] < best["heuristic"], (best, actions)
        g.free()
    finally:
        ctx.set_policy(None)


def torch_rows(rows, n):
    """The first n rows of (depth, parent) host arrays, as check_rows takes them."""
    import torch
    return torch.from_numpy(rows[0][:n]), torch.from_numpy(rows[1][:n])
