"""GPU parity: gr_bfs / gr_sssp through the C ABI against the CPU oracle,
element by element, bit-exact (all arithmetic is integer).  Sizes span many
workgroups and end in ragged tails; every strategy and policy is exercised
(the strategy may change only the time, never the result)."""
import numpy as np
import pytest

import oracle
import paper_1701_01170_amd as gr
from conftest import golden_graph, load_golden
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu

U32MAX = 0xFFFFFFFF
POLICIES = [
    ("heuristic", dict()),
    ("push_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC)),
    ("push_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB)),
    ("push_lb_nolight", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0)),
    ("push_lb_light", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=1 << 30)),
    ("pull_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_TWC)),
    ("pull_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_LB)),
    ("random1", dict(policy=gr.POLICY_RANDOM, policy_seed=1)),
    ("random2", dict(policy=gr.POLICY_RANDOM, policy_seed=2, lb_light_threshold=0)),
    ("chunk512", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                      lb_chunk=512)),
    ("chunk1024", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                       lb_chunk=1024)),
    ("chunk2048", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                       lb_chunk=2048)),
    ("chunk4096", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                       lb_chunk=4096)),
    ("chunk16384", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                        lb_chunk=16384)),
    # iteration control: host round trip per level, and device blocks that
    # stop on a tiny edge bound or run every small push level
    ("dl_off", dict(device_max_edges=-1)),
    ("dl_tiny", dict(device_max_edges=64)),
    ("dl_fixed_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC,
                          device_max_edges=1 << 24)),
    # blocks of device-predicated levels recorded and replayed as hipGraphs
    ("dl_graph", dict(graph_blocks=1)),
    ("dl_graph_twc", dict(graph_blocks=1, policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC,
                          device_max_edges=1 << 24)),
    # launch shapes the autotuner sweeps: workgroup size and TWC tier cut-offs
    ("block128_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                         adv_block=128, device_max_edges=-1)),
    ("block512_lb16384", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB, lb_light_threshold=0,
                              adv_block=512, lb_chunk=16384, device_max_edges=-1)),
    ("block512_light", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB,
                            lb_light_threshold=1 << 30, adv_block=512, device_max_edges=-1)),
    ("block128_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC, adv_block=128,
                          device_max_edges=-1)),
    ("twc_tiers_small", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC, twc_wave_min=4,
                             twc_block_min=9, adv_block=512, device_max_edges=-1)),
    ("twc_tiers_large", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC, twc_wave_min=700,
                             twc_block_min=100000, device_max_edges=-1)),
]
# SSSP also runs with the two-level priority queue: one-distance buckets
# (delta 1), small and large buckets, refills on the host and inside device
# blocks, and a threshold beyond every distance
SSSP_POLICIES = POLICIES + [
    ("pq1", dict(sssp_delta=1)),
    ("pq16", dict(sssp_delta=16)),
    ("pq64_host", dict(sssp_delta=64, device_max_edges=-1)),
    ("pq64_twc_tiny", dict(sssp_delta=64, policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC,
                           device_max_edges=64)),
    ("pq7_light", dict(sssp_delta=7, lb_light_threshold=1 << 30)),
    ("pq_huge", dict(sssp_delta=1 << 30)),
    ("pq16_graph", dict(sssp_delta=16, graph_blocks=1)),
    # every improved vertex kept in the next frontier (the cull of vertices
    # already relaxed with their final distance switched off)
    ("cull_off", dict(sssp_opt_off=gr.SSSP_OPT_CULL)),
    ("bins_off", dict(sssp_opt_off=gr.SSSP_OPT_BINS)),
    ("opts_off", dict(sssp_opt_off=gr.SSSP_OPT_CULL | gr.SSSP_OPT_BINS)),
    ("pq16_cull_off", dict(sssp_delta=16, sssp_opt_off=gr.SSSP_OPT_CULL)),
]


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


def np_of(t):
    return t.cpu().numpy()


# every traversal runs in the caller's numbering (the default) and on the
# degree-renumbered graph
ORDERS = (False, True)


def run_bfs_all(ctx, hg, sources, symmetric=True, policies=POLICIES):
    for keep in ORDERS:
        g = gr.Graph.from_host(ctx, hg, symmetric=symmetric, renumber=keep)
        for s in sources:
            ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, int(s))
            for name, kw in policies:
                d, p, st = gr.bfs(g, int(s), opts=gr.default_opts(**kw))
                msg = f"src={s} policy={name} renumber={keep}"
                np.testing.assert_array_equal(np_of(d), ed, err_msg="depth " + msg)
                np.testing.assert_array_equal(np_of(p), ep, err_msg="parent " + msg)
                assert st["teps_edges"] == oracle.teps_edges(hg.row_offsets, ed >= 0)
                assert st["iterations"] == int(ed.max()) + 1
        g.free()


def run_sssp_all(ctx, hg, source_sets, symmetric=True, policies=SSSP_POLICIES):
    for keep in ORDERS:
        g = gr.Graph.from_host(ctx, hg, symmetric=symmetric, renumber=keep)
        for srcs in source_sets:
            ed, ep = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, srcs)
            for name, kw in policies:
                d, p, st = gr.sssp(g, srcs, opts=gr.default_opts(**kw))
                msg = f"srcs={list(srcs)[:4]} policy={name} renumber={keep}"
                np.testing.assert_array_equal(np_of(d).view(np.uint32), ed, err_msg="dist " + msg)
                np.testing.assert_array_equal(np_of(p), ep, err_msg="pred " + msg)
                assert st["teps_edges"] == oracle.teps_edges(hg.row_offsets, ed != U32MAX)
        g.free()


@pytest.mark.parametrize("name", ["directed7.txt", "undirected_ties8.txt"])
def test_golden(ctx, name):
    fx = load_golden(name)
    hg = golden_graph(fx)
    for keep in ORDERS:
        run_golden(ctx, fx, hg, keep)


def run_golden(ctx, fx, hg, keep):
    g = gr.Graph.from_host(ctx, hg, symmetric=fx["undirected"], renumber=keep)
    for case in fx["bfs"]:
        for pname, kw in POLICIES:
            d, p, _ = gr.bfs(g, case["source"], opts=gr.default_opts(**kw))
            np.testing.assert_array_equal(np_of(d), case["depth"], err_msg=pname)
            np.testing.assert_array_equal(np_of(p), case["parent"], err_msg=pname)
    for case in fx["sssp"]:
        for pname, kw in SSSP_POLICIES:
            d, p, _ = gr.sssp(g, [case["source"]], opts=gr.default_opts(**kw))
            np.testing.assert_array_equal(np_of(d).view(np.uint32).astype(np.int64), case["dist"],
                                          err_msg=pname)
            np.testing.assert_array_equal(np_of(p), case["pred"], err_msg=pname)


def test_rmat14_bfs_all_policies(ctx, rmat14):
    run_bfs_all(ctx, rmat14, gg.sources(rmat14, 6, seed=1000))


def test_rmat14_sssp_all_policies(ctx, rmat14):
    srcs = gg.sources(rmat14, 3, seed=1000)
    run_sssp_all(ctx, rmat14, [[int(s)] for s in srcs] + [srcs.tolist()])


def test_grid_bfs_sssp(ctx):
    hg = gg.add_weights(gg.grid(61, 173), seed=5)
    run_bfs_all(ctx, hg, [0, 61 * 173 // 2 + 17, 61 * 173 - 1])
    run_sssp_all(ctx, hg, [[0], [5000, 9], [61 * 173 - 1]])


def test_er_bfs_sssp(ctx):
    hg = gg.add_weights(gg.erdos_renyi(30001, 6, seed=3), seed=8)
    run_bfs_all(ctx, hg, gg.sources(hg, 3, seed=4))
    run_sssp_all(ctx, hg, [[int(s)] for s in gg.sources(hg, 2, seed=4)])


@pytest.mark.parametrize("lo,hi", [(1, 2), (30000, 140000), (100, 127)])
def test_sssp_distance_mirror(ctx, lo, hi):
    # large frontiers relax through the byte-mark filter, screened by the
    # one-byte distance mirror (ceil(dist / 2^shift), 255 = unknown) once most
    # vertices are reached: weights 1..2 make tight in-edges (predecessor
    # ties) common at quantum 1; weights 30000..140000 quantise by 2^12;
    # weights 100..127 (quantum 2) leave 83-87% of the distances above the
    # 254 quanta the mirror holds, so most of its entries saturate
    hg = gg.add_weights(gg.erdos_renyi(30001, 8, seed=11), seed=12, lo=lo, hi=hi)
    run_sssp_all(ctx, hg, [[int(s)] for s in gg.sources(hg, 2, seed=13)])


@pytest.mark.parametrize("lo,hi", [(0, 3), (1, 64)])
def test_sssp_cull_of_relaxed_vertices(ctx, lo, hi):
    # Large R-MAT levels relax through the byte-mark filter, whose compaction
    # drops vertices whose edges already went out with their final distance
    # and lists the rest in bins of distance: results identical with either
    # refinement on or off (also with zero weights, where distance 0 and ties
    # are common, and with the priority queue), and fewer edges relaxed with
    # them on.  A vertex can only be dropped when its distance fell before a
    # chunk of its row was staged, i.e. in levels with more chunks than
    # resident workgroups: hence 1024-edge chunks at scale 18.
    hg = gg.add_weights(gg.rmat(18, 16, seed=7), seed=17, lo=lo, hi=hi)
    lb = dict(lb_chunk=1024, lb_light_threshold=0)
    offs = (0, gr.SSSP_OPT_CULL, gr.SSSP_OPT_BINS, gr.SSSP_OPT_CULL | gr.SSSP_OPT_BINS)
    for keep in ORDERS:
        g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=keep)
        inspected = {off: 0 for off in offs}
        for s in gg.sources(hg, 3, seed=5):
            ed, ep = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [int(s)])
            for off in offs:
                for extra in (lb, dict(), dict(sssp_delta=8, **lb), dict(adv_block=512),
                              dict(lb_light_threshold=1 << 30), dict(device_max_edges=-1, **lb)):
                    d, p, st = gr.sssp(g, [int(s)], opts=gr.default_opts(sssp_opt_off=off, **extra))
                    msg = f"src={s} sssp_opt_off={off} {extra} renumber={keep}"
                    np.testing.assert_array_equal(np_of(d).view(np.uint32), ed, err_msg="dist " + msg)
                    np.testing.assert_array_equal(np_of(p), ep, err_msg="pred " + msg)
                    if extra is lb:
                        inspected[off] += st["inspected_edges"]
        both = gr.SSSP_OPT_CULL | gr.SSSP_OPT_BINS
        assert inspected[0] < inspected[both], inspected
        assert inspected[gr.SSSP_OPT_BINS] < inspected[both], inspected
        g.free()


def test_unsorted_input_is_sorted_on_ingest(ctx, rmat14):
    hg = rmat14
    rng = np.random.default_rng(0)
    C = hg.col_indices.copy()
    W = hg.weights.copy()
    R = hg.row_offsets
    for v in rng.choice(hg.n_vertices, 500, replace=False):
        a, b = R[v], R[v + 1]
        perm = rng.permutation(b - a)
        C[a:b] = C[a:b][perm]
        W[a:b] = W[a:b][perm]
    shuffled = gg.HostGraph(R.copy(), C, W)
    for keep in ORDERS:
        # export gives the sorted CSR in the caller's ids, renumbered or not
        g = gr.Graph.from_host(ctx, shuffled, renumber=keep)
        assert g.resorted
        R2, C2, W2 = g.export()
        np.testing.assert_array_equal(np_of(R2), hg.row_offsets)
        np.testing.assert_array_equal(np_of(C2), hg.col_indices)
        np.testing.assert_array_equal(np_of(W2).view(np.uint32), hg.weights)
        g.free()
    srcs = gg.sources(hg, 2, seed=9)
    run_bfs_all(ctx, shuffled, srcs)
    run_sssp_all(ctx, shuffled, [[int(srcs[0])]])


def test_long_unsorted_rows(ctx):
    # a star whose centre list (5000 > LDS sort size) arrives reversed
    n = 5001
    edges = [(0, i) for i in range(n - 1, 0, -1)] + [(i, 0) for i in range(1, n)]
    w = [(i * 7) % 64 + 1 for i in range(len(edges))]
    hg = gg.from_edges(n, edges, w)
    g = gr.Graph.from_host(ctx, hg)
    assert g.resorted
    _, C2, _ = g.export()
    np.testing.assert_array_equal(np_of(C2)[:n - 1], np.arange(1, n))
    g.free()
    run_bfs_all(ctx, hg, [0, 17])
    run_sssp_all(ctx, hg, [[0], [17]])


def test_directed_random(ctx):
    rng = np.random.default_rng(3)
    V = 20000
    e = rng.integers(0, V, size=(120000, 2))
    w = rng.integers(1, 65, size=120000)
    hg = gg.sort_adjacency(gg.from_edges(V, e, w))
    srcs = rng.integers(0, V, size=3)
    run_bfs_all(ctx, hg, srcs, symmetric=False)
    run_sssp_all(ctx, hg, [[int(s)] for s in srcs], symmetric=False)


def test_degenerate_graphs(ctx):
    # one vertex, no edges
    hg = gg.HostGraph(np.array([0, 0], np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint32))
    run_bfs_all(ctx, hg, [0])
    run_sssp_all(ctx, hg, [[0]])
    # isolated source inside a bigger graph, self-loops and duplicate edges
    hg = gg.from_edges(6, [(1, 2), (2, 1), (2, 2), (2, 3), (3, 2), (2, 3), (3, 2), (4, 4)],
                       [3, 3, 1, 9, 9, 2, 2, 1])
    hg = gg.sort_adjacency(hg)
    run_bfs_all(ctx, hg, [0, 1, 4], symmetric=False)
    run_sssp_all(ctx, hg, [[0], [1], [1, 4]], symmetric=False)
    # zero weights: ties at distance 0, sources keep pred -1
    hg = gg.from_edges(5, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)], [0, 0, 0, 0, 5], symmetric=True)
    hg = gg.sort_adjacency(hg)
    run_sssp_all(ctx, hg, [[0], [0, 2], [4]])


def test_hub_frontier_spans_many_chunks(ctx):
    # two hubs of degree 60000 -> frontier segments far longer than one LB chunk
    n = 60002
    edges = [(0, i) for i in range(2, n)] + [(1, i) for i in range(2, n)]
    hg = gg.add_weights(gg.sort_adjacency(gg.from_edges(n, edges, symmetric=True)), seed=2)
    run_bfs_all(ctx, hg, [0, 5])
    run_sssp_all(ctx, hg, [[0], [5]])


def test_errors_on_device(ctx, rmat14):
    g = gr.Graph.from_host(ctx, rmat14)
    with pytest.raises(gr.GrError) as ei:
        gr.bfs(g, rmat14.n_vertices)
    assert ei.value.code == gr.GR_EINVAL
    with pytest.raises(gr.GrError) as ei:
        gr.sssp(g, [-1])
    assert ei.value.code == gr.GR_EINVAL
    g2 = gr.Graph.from_csr(ctx, rmat14.row_offsets, rmat14.col_indices)
    with pytest.raises(gr.GrError) as ei:
        gr.sssp(g2, [0])
    assert ei.value.code == gr.GR_EINVAL
    big = gg.from_edges(3, [(0, 1), (1, 2)], [0xF0000000, 0x20000000])
    g3 = gr.Graph.from_host(ctx, big, symmetric=False)
    with pytest.raises(gr.GrError) as ei:
        gr.sssp(g3, [0])
    assert ei.value.code == gr.GR_ERANGE


def test_device_input_csr(ctx, rmat14):
    import torch
    R = torch.from_numpy(rmat14.row_offsets).cuda()
    C = torch.from_numpy(rmat14.col_indices).cuda()
    W = torch.from_numpy(rmat14.weights.view(np.int32)).cuda()
    g = gr.Graph.from_csr(ctx, R, C, W)
    assert g.n_edges == rmat14.n_edges and g.max_degree == rmat14.degrees().max()
    s = int(gg.sources(rmat14, 1)[0])
    d, p, _ = gr.bfs(g, s)
    ed, ep = oracle.bfs(rmat14.row_offsets, rmat14.col_indices, s)
    np.testing.assert_array_equal(np_of(d), ed)
    np.testing.assert_array_equal(np_of(p), ep)
    bad = C.clone()
    bad[7] = rmat14.n_vertices
    with pytest.raises(gr.GrError) as ei:
        gr.Graph.from_csr(ctx, R, bad, W)
    assert ei.value.code == gr.GR_EINVAL


def test_max_iterations_stops_early(ctx, rmat14):
    g = gr.Graph.from_host(ctx, rmat14)
    s = int(gg.sources(rmat14, 1)[0])
    ed, _ = oracle.bfs(rmat14.row_offsets, rmat14.col_indices, s)
    d, _, st = gr.bfs(g, s, opts=gr.default_opts(max_iterations=2))
    exp = np.where(ed <= 2, ed, -1)
    np.testing.assert_array_equal(np_of(d), exp)
    assert st["iterations"] == 2


@pytest.mark.parametrize("dme", [0, -1, 1 << 24])
def test_trace_records(ctx, rmat14, dme):
    g = gr.Graph.from_host(ctx, rmat14)
    s = int(gg.sources(rmat14, 1)[0])
    ed, _ = oracle.bfs(rmat14.row_offsets, rmat14.col_indices, s)
    prof = oracle.level_profile(rmat14.row_offsets, ed)
    cap = 64
    buf = (gr.LevelTrace * cap)()
    o = gr.default_opts(trace=buf, trace_capacity=cap, device_max_edges=dme)
    d, p, _ = gr.bfs(g, s, opts=o)
    _, ep = oracle.bfs(rmat14.row_offsets, rmat14.col_indices, s)
    np.testing.assert_array_equal(np_of(d), ed)
    np.testing.assert_array_equal(np_of(p), ep)
    assert o.trace_count == len(prof)
    for t, ref in zip(buf[:o.trace_count], prof):
        assert (t.level, t.n_f, t.m_f, t.n_u, t.m_u, t.max_deg_f) == (
            ref["level"], ref["n_f"], ref["m_f"], ref["n_u"], ref["m_u"], ref["maxdeg_f"])
        assert t.step_us > 0
    kernels = {t.kernel for t in buf[:o.trace_count]}
    assert (6 in kernels) == (dme != -1), kernels


@pytest.mark.parametrize("steps_off", [0, 1])
@pytest.mark.parametrize("delta", [0, 16])
@pytest.mark.parametrize("dme", [0, -1])
def test_traced_sssp_outputs(ctx, rmat14, dme, delta, steps_off):
    """Tracing takes its own paths (event records around every advance
    kernel, the block logs of device-predicated levels published with the
    control block); the traced SSSP must still match the oracle element by
    element.  With trace_steps_off only the advance kernels are timed: step
    times stay 0 outside device-predicated blocks."""
    g = gr.Graph.from_host(ctx, rmat14)
    cap = 256
    buf = (gr.LevelTrace * cap)()
    for s in gg.sources(rmat14, 2, seed=1000):
        o = gr.default_opts(trace=buf, trace_capacity=cap, device_max_edges=dme, sssp_delta=delta,
                            trace_steps_off=steps_off)
        d, p, st = gr.sssp(g, [int(s)], opts=o)
        ed, ep = oracle.sssp(rmat14.row_offsets, rmat14.col_indices, rmat14.weights, [int(s)])
        np.testing.assert_array_equal(np_of(d).view(np.uint32), ed)
        np.testing.assert_array_equal(np_of(p), ep)
        assert 0 < o.trace_count <= cap
        recs = buf[:o.trace_count]
        assert all(t.kernel_us > 0 for t in recs)
        if steps_off:
            assert all(t.step_us == 0 for t in recs if t.kernel != 6)
        else:
            assert all(t.step_us > 0 for t in recs)
    g.free()


@pytest.mark.parametrize("max_it", [1, 3, 4, 37, 100])
def test_device_blocks_respect_max_iterations(ctx, max_it):
    """Long chains of small levels (a thin grid) run in device blocks of
    4, 8, 16, ... levels; a level cap that falls inside a block still stops
    exactly there."""
    hg = gg.add_weights(gg.grid(7, 301), seed=9)
    g = gr.Graph.from_host(ctx, hg)
    ed, _ = oracle.bfs(hg.row_offsets, hg.col_indices, 0)
    d, _, st = gr.bfs(g, 0, opts=gr.default_opts(max_iterations=max_it))
    np.testing.assert_array_equal(np_of(d), np.where(ed <= max_it, ed, -1))
    assert st["iterations"] == min(max_it, int(ed.max()) + 1)
    edist, _ = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [0])
    for kw in (dict(), dict(sssp_delta=32), dict(sssp_delta=3, device_max_edges=-1)):
        dist, _, st = gr.sssp(g, [0], opts=gr.default_opts(**kw))
        np.testing.assert_array_equal(np_of(dist).view(np.uint32), edist, err_msg=str(kw))
    g.free()


def test_block_graphs_replayed_between_eager_runs(ctx):
    """Instantiated block graphs are kept in the context and updated with each
    block's arguments: replays alternate with eager runs (and host
    synchronisations) and every result must equal the oracle."""
    import torch
    hg = gg.add_weights(gg.grid(90, 70), seed=3)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    for rnd, s in enumerate([0, 3150, 6299, 77, 0]):
        ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, s)
        edist, epred = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s])
        for graph in (1, 0, 1):
            o = gr.default_opts(graph_blocks=graph)
            d, p, st = gr.bfs(g, s, opts=o)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(np_of(d), ed, err_msg=f"bfs round {rnd} graph {graph}")
            np.testing.assert_array_equal(np_of(p), ep, err_msg=f"bfs round {rnd} graph {graph}")
            dist, pred, _ = gr.sssp(g, [s], opts=gr.default_opts(graph_blocks=graph, sssp_delta=32 * rnd))
            np.testing.assert_array_equal(np_of(dist).view(np.uint32), edist)
            np.testing.assert_array_equal(np_of(pred), epred)
    g.free()
