"""GPU parity of betweenness centrality (gr_bc; paper Sec. 6, Brandes's two
passes) against the float64 CPU oracle, element by element.

Tolerance: both sides compute in IEEE double.  Path counts are integers and
exact while below 2^53, so sigma is compared exactly on these graphs.  The
dependencies are sums of positive terms taken in a different order (the GPU
adds them with atomics or per-row reductions, the oracle in adjacency order); each term carries a
few roundings and the sums chain over the levels, so the relative error stays
below (levels + largest degree) * 4 * 2^-53 < 1e-9 here; the test allows
rtol 1e-9 against max(1, |expected|)."""
import math

import numpy as np
import pytest

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu

RTOL = 1e-9
POLICIES = [
    ("heuristic", dict()),
    ("push_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_TWC)),
    ("lb_nolight", dict(lb_light_threshold=0)),
    ("lb_chunk512", dict(lb_light_threshold=0, lb_chunk=512)),
    ("light_only", dict(lb_light_threshold=1 << 30)),
    ("twc_levels", dict(lb_min_avg_degree=math.inf)),
    ("pull_lb", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_LB)),
    # per-pass directions (forward | backward << 2): both pushed (fp64 atomics
    # onto the other end of each edge), both pulled, and mixed
    ("push_both", dict(bc_dir=gr.BC_DIR_PUSH | gr.BC_DIR_PUSH << 2)),
    ("pull_both", dict(bc_dir=gr.BC_DIR_PULL | gr.BC_DIR_PULL << 2)),
    ("push_fwd_twc", dict(bc_dir=gr.BC_DIR_PUSH | gr.BC_DIR_PULL << 2,
                          lb_min_avg_degree=math.inf)),
    # pull chunks of 16384 edges take four batches per workgroup and, on rows
    # of a few edges, more rows than one LDS stage holds
    ("pull_chunk16384", dict(bc_dir=gr.BC_DIR_PULL | gr.BC_DIR_PULL << 2, lb_chunk=16384)),
    ("push_bwd_chunk512", dict(bc_dir=gr.BC_DIR_AUTO | gr.BC_DIR_PUSH << 2, lb_chunk=512)),
    # the knobs the autotuner stores for BC on R-MAT 22 (the benchmark's setting)
    ("tuned_like", dict(lb_light_threshold=0, lb_chunk=1024, do_a=1 / 64, do_b=1 / 64,
                        device_max_edges=1 << 20)),
]
PUSH_PULL = [POLICIES[0], POLICIES[7], POLICIES[8], POLICIES[10], POLICIES[12]]


@pytest.fixture(scope="module")
def ctx():
    return gr.Context(0)


def close(got, expect, msg=""):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - expect) / np.maximum(1.0, np.abs(expect))
    i = int(np.argmax(err))
    assert err[i] <= RTOL, f"{msg} v={i} got={got[i]!r} expect={expect[i]!r} rel={err[i]:.3g}"


def check_graph(ctx, hg, source_sets, policies=POLICIES, renumber=(False, True)):
    for keep in renumber:
        g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=keep)
        for srcs in source_sets:
            eb, es = oracle.bc(hg.row_offsets, hg.col_indices, srcs, want_sigma=len(srcs) == 1)
            for name, kw in policies:
                msg = f"srcs={list(srcs)[:4]} policy={name} renumber={keep}"
                b, sig, st = gr.bc(g, srcs, want_sigma=len(srcs) == 1, opts=gr.default_opts(**kw))
                close(b.cpu().numpy(), eb, "bc " + msg)
                if es is not None and es.max() < 2.0 ** 53:
                    np.testing.assert_array_equal(sig.cpu().numpy(), es, err_msg="sigma " + msg)
                assert st["teps_edges"] > 0 or hg.n_edges == 0
        g.free()


def test_rmat14(ctx, rmat14):
    s = gg.sources(rmat14, 4, seed=1000)
    check_graph(ctx, rmat14, [[int(s[0])], s.tolist()])


def test_grid_sigma_closed_form(ctx):
    rows, cols = 23, 29
    hg = gg.grid(rows, cols)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    _, sig, _ = gr.bc(g, [0], want_sigma=True)
    r, c = np.divmod(np.arange(rows * cols), cols)
    expect = np.array([math.comb(int(a + b), int(a)) for a, b in zip(r, c)], dtype=np.float64)
    np.testing.assert_array_equal(sig.cpu().numpy(), expect)
    g.free()
    check_graph(ctx, hg, [[0], [rows * cols // 2 + 3], [5, 77, 400]])


def test_er_and_union(ctx):
    er = gg.erdos_renyi(20001, 6, seed=3)
    check_graph(ctx, er, [[int(x) for x in gg.sources(er, 3, seed=4)]], policies=PUSH_PULL)
    parts = [gg.rmat(s, 8, seed=10 + s) for s in (7, 9, 10)]
    u, voff = gg.disjoint_union(parts)
    check_graph(ctx, u, [[int(voff[0]) + 1, int(voff[1]) + 2, int(voff[2]) + 3]],
                policies=POLICIES[:2])


def test_closed_forms(ctx):
    # path longer than the level histogram kept in LDS (4096 levels)
    n = 5000
    path = gg.from_edges(n, [(i, i + 1) for i in range(n - 1)], None, symmetric=True)
    g = gr.Graph.from_host(ctx, path, symmetric=True)
    b, sig, st = gr.bc(g, [0], want_sigma=True)
    v = np.arange(n)
    np.testing.assert_array_equal(b.cpu().numpy(), np.where(v == 0, 0.0, n - 1 - v))
    np.testing.assert_array_equal(sig.cpu().numpy(), np.ones(n))
    assert st["iterations"] == n
    g.free()
    # star: from every vertex, the centre carries n (n - 1)
    k = 300
    star = gg.from_edges(k + 1, [(0, i) for i in range(1, k + 1)], None, symmetric=True)
    g = gr.Graph.from_host(ctx, star, symmetric=True)
    b, _, _ = gr.bc(g, np.arange(k + 1))
    bn = b.cpu().numpy()
    assert bn[0] == k * (k - 1) and np.all(bn[1:] == 0)
    g.free()
    # complete bipartite K_{m,n}
    m, nb = 6, 500
    kb = gg.from_edges(m + nb, [(a, m + j) for a in range(m) for j in range(nb)], None,
                       symmetric=True)
    g = gr.Graph.from_host(ctx, kb, symmetric=True)
    b, _, _ = gr.bc(g, np.arange(m + nb))
    bn = b.cpu().numpy()
    np.testing.assert_allclose(bn[:m], nb * (nb - 1) / m, rtol=RTOL)
    np.testing.assert_allclose(bn[m:], m * (m - 1) / nb, rtol=RTOL)
    g.free()


def test_isolated_source_and_errors(ctx):
    hg = gg.from_edges(10, [(1, 2), (2, 3)], None, symmetric=True)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    b, sig, st = gr.bc(g, [0], want_sigma=True)
    assert np.all(b.cpu().numpy() == 0)
    np.testing.assert_array_equal(sig.cpu().numpy(), np.eye(1, 10, 0).ravel())
    with pytest.raises(gr.GrError) as ei:
        gr.bc(g, [1, 2], want_sigma=True)
    assert ei.value.code == gr.GR_EINVAL
    for bad in (3, 3 << 2, -1, 16):  # each pass takes AUTO, PUSH or PULL
        with pytest.raises(gr.GrError) as ei:
            gr.bc(g, [1], opts=gr.default_opts(bc_dir=bad))
        assert ei.value.code == gr.GR_EINVAL
    g.free()
    d = gr.Graph.from_host(ctx, hg, symmetric=False)
    with pytest.raises(gr.GrError) as ei:
        gr.bc(d, [1])
    assert ei.value.code == gr.GR_EUNSUPPORTED
    d.free()


def test_rmat20_two_sources(ctx):
    hg = gg.rmat(20, 16, seed=1)
    srcs = [int(x) for x in gg.sources(hg, 2, seed=3000)]
    print(f"bc rmat20 V={hg.n_vertices} E={hg.n_edges} sources={srcs}", flush=True)
    check_graph(ctx, hg, [srcs], policies=[POLICIES[0], POLICIES[7], POLICIES[8], POLICIES[12]],
                renumber=(False, True))
