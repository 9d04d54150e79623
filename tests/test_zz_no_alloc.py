"""gr_bfs_static (BFS with its working arrays in the library's static device
workspace, for callers that cannot allocate) against gr_bfs through the C ABI:
bit-exact depths and parents on two calls in a row, the second on a smaller
graph, plus renumbered / directed / traced / parent-less variants, the size
limit, and the absence of device allocations inside the call."""
import numpy as np
import pytest

import oracle
import paper_1701_01170_amd as gr
from paper_1701_01170_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def _run_both(g, src, opts_kw=None, want_parent=True):
    import torch
    kw = dict(opts_kw or {})
    d0, p0, s0 = gr.bfs(g, src, want_parent=want_parent, opts=gr.default_opts(**kw))
    V = g.n_vertices
    d1 = torch.full((V,), 12345, dtype=torch.int32, device="cuda")
    p1 = torch.full((V,), 12345, dtype=torch.int32, device="cuda") if want_parent else None
    s1 = gr.bfs_static(g, src, (d1, p1), opts=gr.default_opts(**kw))
    torch.cuda.synchronize()
    return (d0, p0, s0), (d1, p1, s1)


def _check_same(a, b, hg, src):
    (d0, p0, s0), (d1, p1, s1) = a, b
    dn0, dn1 = d0.cpu().numpy(), d1.cpu().numpy()
    assert np.array_equal(dn0, dn1), f"depth differs at {np.flatnonzero(dn0 != dn1)[:8]}"
    ed, ep = oracle.bfs(hg.row_offsets, hg.col_indices, src)
    assert np.array_equal(dn1, ed)
    if p0 is not None:
        pn0, pn1 = p0.cpu().numpy(), p1.cpu().numpy()
        assert np.array_equal(pn0, pn1), f"parent differs at {np.flatnonzero(pn0 != pn1)[:8]}"
        assert np.array_equal(pn1, ep)
    assert s0["iterations"] == s1["iterations"]
    assert s0["teps_edges"] == s1["teps_edges"]


def test_two_calls_in_a_row_second_smaller():
    ctx = gr.Context(0)
    big = gg.rmat(18, 16, seed=3)
    small = gg.rmat(11, 8, seed=4)
    gb = gr.Graph.from_host(ctx, big, symmetric=True)
    gs = gr.Graph.from_host(ctx, small, symmetric=True)
    sb = int(gg.sources(big, 1, seed=1003)[0])
    ss = int(gg.sources(small, 1, seed=1004)[0])
    print(f"static bfs: rmat18 V={big.n_vertices} E={big.n_edges} src={sb}", flush=True)
    _check_same(*_run_both(gb, sb), big, sb)
    print(f"static bfs: rmat11 V={small.n_vertices} E={small.n_edges} src={ss}", flush=True)
    _check_same(*_run_both(gs, ss), small, ss)
    # and back to the large one: nothing the small call left may leak in
    _check_same(*_run_both(gb, sb), big, sb)
    gb.free()
    gs.free()
    ctx.close()


@pytest.mark.parametrize("name,kw", [
    ("pull_twc", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PULL_TWC)),
    ("push_lb_nolight", dict(policy=gr.POLICY_FIXED, fixed_action=gr.PUSH_LB,
                             lb_light_threshold=0)),
    ("dl_off", dict(device_max_edges=-1)),
])
def test_policies(name, kw):
    ctx = gr.Context(0)
    hg = gg.rmat(16, 16, seed=5)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    src = int(gg.sources(hg, 1, seed=1005)[0])
    print(f"static bfs: {name} rmat16 src={src}", flush=True)
    _check_same(*_run_both(g, src, kw), hg, src)
    g.free()
    ctx.close()


def _traced(g, src, static):
    import torch
    cap = 256
    tr = (gr.LevelTrace * cap)()
    o = gr.default_opts(trace=tr, trace_capacity=cap)
    V = g.n_vertices
    if static:
        d = torch.empty(V, dtype=torch.int32, device="cuda")
        p = torch.empty(V, dtype=torch.int32, device="cuda")
        s = gr.bfs_static(g, src, (d, p), opts=o)
    else:
        d, p, s = gr.bfs(g, src, opts=o)
    torch.cuda.synchronize()
    recs = [(tr[i].level, tr[i].action, tr[i].n_f, tr[i].m_f, tr[i].n_next)
            for i in range(min(o.trace_count, cap))]
    return (d, p, s), recs


def test_traced_renumbered_directed_and_no_parent():
    ctx = gr.Context(0)
    hg = gg.rmat(15, 16, seed=6)
    src = int(gg.sources(hg, 1, seed=1006)[0])
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    print(f"static bfs: renumbered rmat15 src={src}", flush=True)
    _check_same(*_run_both(g, src), hg, src)
    print("static bfs: traced", flush=True)
    a, ra = _traced(g, src, static=False)
    b, rb = _traced(g, src, static=True)
    _check_same(a, b, hg, src)
    assert len(ra) > 0 and ra == rb
    print("static bfs: no parent", flush=True)
    _check_same(*_run_both(g, src, want_parent=False), hg, src)
    g.free()
    # directed graph (push only)
    edges = np.array([(i, (7 * i + 3) % 500) for i in range(500)] +
                     [(i, i + 1) for i in range(499)], dtype=np.int64)
    dg = gg.from_edges(500, edges, None, symmetric=False)
    gd = gr.Graph.from_host(ctx, dg, symmetric=False)
    print("static bfs: directed", flush=True)
    _check_same(*_run_both(gd, 0), dg, 0)
    gd.free()
    ctx.close()


def test_too_large_is_rejected_before_device_work():
    import torch
    ctx = gr.Context(0)
    V = 2_400_000  # a path: about 29 bytes per vertex exceed the 64 MiB workspace
    R = np.concatenate([[0, 1], 1 + 2 * np.arange(1, V - 1), [2 * (V - 1)]]).astype(np.int32)
    mids = np.stack([np.arange(0, V - 2), np.arange(2, V)], axis=1).ravel()
    C = np.concatenate([[1], mids, [V - 2]]).astype(np.int32)
    assert C.shape[0] == R[-1]
    g = gr.Graph.from_csr(ctx, R, C, None, symmetric=True)
    depth = torch.full((V,), 7, dtype=torch.int32, device="cuda")
    print("static bfs: too large", flush=True)
    with pytest.raises(gr.GrError) as ei:
        gr.bfs_static(g, 0, (depth, None))
    assert ei.value.code == gr.GR_ERANGE
    assert "static workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert int((depth != 7).sum()) == 0  # nothing ran
    g.free()
    # the context and the workspace still work afterwards
    small = gg.rmat(10, 8, seed=7)
    gs = gr.Graph.from_host(ctx, small, symmetric=True)
    s = int(gg.sources(small, 1, seed=1007)[0])
    _check_same(*_run_both(gs, s), small, s)
    gs.free()
    ctx.close()


def test_no_device_allocation_inside_the_call():
    """The static call leaves free device memory unchanged, where gr_bfs on a
    fresh context grows its pool by several MiB (so the probe can see it)."""
    import torch
    ctx = gr.Context(0)
    hg = gg.rmat(18, 16, seed=8)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    src = int(gg.sources(hg, 1, seed=1008)[0])
    V = hg.n_vertices
    d = torch.empty(V, dtype=torch.int32, device="cuda")
    p = torch.empty(V, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    gr.bfs_static(g, src, (d, p))
    gr.bfs_static(g, src, (d, p))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    gr.bfs(g, src, out=(d, p))
    torch.cuda.synchronize()
    free2, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (1 << 20), (free0, free1)
    assert free1 - free2 > (4 << 20), (free1, free2)  # the pool path does allocate
    g.free()
    ctx.close()
