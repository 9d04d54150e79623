"""Benchmark: BFS and SSSP on an undirected R-MAT graph of scale 22 (edge
factor 16, a=0.57 b=0.19 c=0.19 d=0.05, uint32 weights uniform in 1..64),
on one MI355X.

A step is one pass of the traversal hot path over the resident graph: a
direction-optimising BFS (depths + canonical parents) and an SSSP (distances +
canonical predecessors) from the same seeded source, each choosing its advance
strategy per iteration with the fixed-threshold heuristic of the paper (library
defaults).  The graph is generated on the host and uploaded before the timed
region.  Throughput is GTEPS = (sum over the step's traversals of the degrees
of the reached vertices) / step time, the paper's TEPS convention (Sec. 7,
measurement methodology).

The timed steps run with per-iteration tracing on, so every advance kernel is
bracketed by HIP events on the traversal's stream; `roofline` divides the
algorithmic bytes of the dominant advance kernel by its event-timed duration.
`traffic` comes from committed rocprofv3 FETCH_SIZE/WRITE_SIZE summaries
(profiles/traffic_*.json) when they were taken on the current kernel source,
else null.  `cpu_baseline` times the CPU oracle (single thread) on BFS + SSSP pairs
of the same workload (about 10 s of CPU work).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1701_01170_amd.rocprof_summary import kernel_source_hash  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {
    ("bfs", 0): "k_push_twc<BfsVisit>", ("bfs", 1): "k_push_light<BfsVisit>",
    ("bfs", 2): "k_push_lb<BfsVisit>", ("bfs", 3): "k_push_lb<BfsMark>",
    ("bfs", 4): "k_bfs_pull_bm<1>", ("bfs", 5): "k_bfs_pull_bm<4>",
    ("sssp", 0): "k_push_twc<SsspVisit>", ("sssp", 1): "k_push_light<SsspVisit>",
    ("sssp", 2): "k_push_lb<SsspVisit>",
    ("bfs", 6): "k_dstep<BfsVisit>", ("sssp", 6): "k_dstep<SsspVisit>",
    ("sssp", 7): "k_sssp_pq_refill",
    ("sssp", 8): "k_push_twc<SsspMark>", ("sssp", 9): "k_push_light<SsspMark>",
    ("sssp", 10): "k_push_lb<SsspMark>",
}


def algorithmic_bytes(kind: str, kernel: int, n_f: int, m_f: int, n_next: int) -> float | None:
    """Bytes the method must move for one advance launch:
    SSSP relax: per edge 4 B column + 4 B weight + 8 B packed atomic-min of the
      target's (dist, pred) key; per frontier vertex 4 B id + 8 B row offsets;
      per output vertex 4 B queue entry.
    BFS push: per edge 4 B column (the visited test is one bit, cache
      resident); per frontier vertex 12 B; per new vertex 4 B depth + 4 B
      parent + 4 B queue entry."""
    if kind == "sssp" and kernel != 7:
        return 16.0 * m_f + 12.0 * n_f + 4.0 * n_next
    if kind == "bfs" and kernel in (0, 1, 2, 3, 6):
        return 4.0 * m_f + 12.0 * n_f + 12.0 * n_next
    return None


def headline_opts(gr, g, cap: int = 4096):
    """The timed configuration of the headline step: the heuristic policy with
    the knobs the autotuner stored for this graph's class and size (paper
    defaults when none are stored), and per-iteration tracing into host
    buffers of `cap` records.  Returns (bfs opts, sssp opts, bfs trace,
    sssp trace); the trace buffers must outlive the opts."""
    from paper_1701_01170_amd import autotune
    tb = (gr.LevelTrace * cap)()
    ts = (gr.LevelTrace * cap)()
    ob = autotune.tuned_opts(g, "bfs", trace=tb, trace_capacity=cap)
    os_ = autotune.tuned_opts(g, "sssp", trace=ts, trace_capacity=cap)
    return ob, os_, tb, ts


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the grid, batched and learned-policy comparisons")
    ap.add_argument("--large", action="store_true",
                    help="instead of the headline, run the largest workload: R-MAT scale 25, "
                         "16-source batched BFS and 16 SSSP runs")
    return ap.parse_args()


def large(args, gr, gg, torch):
    """R-MAT scale 25 (edge factor 16, ~1.07B directed edges, uint32 weights
    1..64) resident in HBM: one 16-source batched BFS and 16 single-source SSSP
    runs back to back, under the learned selector when trained weights exist
    (else the heuristic).  Prints its own JSON line."""
    from paper_1701_01170_amd import autotune, selector
    t0 = time.time()
    hg = gg.add_weights(gg.rmat(25, 16, seed=1), seed=101)
    print(f"# generated {hg.name}: V={hg.n_vertices} E={hg.n_edges} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ctx = gr.Context(0)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    srcs = gg.sources(hg, 16, seed=1000).astype(np.int32)
    V = hg.n_vertices
    del hg
    policy = "heuristic"
    if os.path.exists(selector.WEIGHTS):
        ctx.set_policy(np.load(selector.WEIGHTS))
        policy = "learned"
    kw = {"policy": gr.POLICY_LEARNED} if policy == "learned" else {}
    depth = torch.empty((16, V), dtype=torch.int32, device="cuda")
    parent = torch.empty((16, V), dtype=torch.int32, device="cuda")
    om = autotune.tuned_opts(g, "bfs_multi")
    gr.bfs_multi(g, srcs[:2], opts=om, out=(depth[:2], parent[:2]))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mb = gr.bfs_multi(g, srcs, opts=om, out=(depth, parent))[2]
    torch.cuda.synchronize()
    bfs_wall = time.perf_counter() - t0
    del depth, parent
    dist = torch.empty(V, dtype=torch.int32, device="cuda")
    pred = torch.empty(V, dtype=torch.int32, device="cuda")
    os_ = autotune.tuned_opts(g, "sssp", **kw)
    gr.sssp(g, [int(srcs[0])], opts=os_, out=(dist, pred))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for s in srcs:
        steps.append(gr.sssp(g, [int(s)], opts=os_, out=(dist, pred))[2])
    torch.cuda.synchronize()
    sssp_wall = time.perf_counter() - t0
    teps = mb["teps_edges"] + sum(st["teps_edges"] for st in steps)
    wall = bfs_wall + sssp_wall
    out = {
        "metric": "GTEPS BFS/SSSP RMAT-25, 16-source batched BFS + 16 SSSP",
        "value": round(teps / wall / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
        "ms_per_step": round(wall * 1e3, 3), "higher_is_better": True, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat_s25_e16, int32 CSR, uint32 weights 1..64; gr_bfs_multi with 16 "
                               "sources + 16 gr_sssp runs", "policy": policy,
                   "n_vertices": V, "n_edges": g.n_edges},
        "breakdown": {"bfs_multi16_ms": round(mb["device_ms"], 3),
                      "bfs_multi16_gteps_device": _gteps(mb["teps_edges"], mb["device_ms"]),
                      "sssp16_ms": round(sum(st["device_ms"] for st in steps), 3),
                      "sssp16_gteps_device": _gteps(sum(st["teps_edges"] for st in steps),
                                                    sum(st["device_ms"] for st in steps))},
    }
    print(json.dumps(out))


def _gteps(teps: float, ms: float) -> float | None:
    return round(teps / (ms * 1e-3) / 1e9, 3) if ms > 0 else None


def extras(gr, gg, ctx, torch, log):
    """Comparison workloads reported next to the headline (device-event time):
    the 2048 x 2048 grid (high diameter, small frontiers), 64-source batched BFS
    on R-MAT scale 20 against 64 single-source runs, 256 small R-MAT graphs in
    one disjoint-union SSSP against 256 separate runs, and (when trained
    weights are present) the learned selector against the heuristic on the
    R-MAT scale 22 workload (filled in by the caller)."""
    from paper_1701_01170_amd import autotune
    out = {}
    # grid
    hg = gg.add_weights(gg.grid(2048, 2048), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    s = int(gg.sources(hg, 1, seed=1000)[0])
    row = {}
    for label, kw in (("device_blocks", {}), ("host_loop", {"device_max_edges": -1})):
        ob = autotune.tuned_opts(g, "bfs", **kw)
        os_ = autotune.tuned_opts(g, "sssp", **kw)
        gr.bfs(g, s, opts=ob)
        b = gr.bfs(g, s, opts=ob)[2]
        t = gr.sssp(g, [s], opts=os_)[2]
        row[label] = {"bfs_ms": round(b["device_ms"], 3), "bfs_gteps": _gteps(b["teps_edges"], b["device_ms"]),
                      "bfs_iterations": b["iterations"], "sssp_ms": round(t["device_ms"], 3),
                      "sssp_gteps": _gteps(t["teps_edges"], t["device_ms"]), "sssp_iterations": t["iterations"]}
    out["grid_2048x2048"] = row
    g.free()
    del hg
    log("# grid done")
    # 64-source batched BFS, R-MAT scale 20
    hg = gg.rmat(20, 16, seed=1)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    srcs = gg.sources(hg, 64, seed=2000).astype(np.int32)
    ob = autotune.tuned_opts(g, "bfs")
    V = hg.n_vertices
    depth = torch.empty((64, V), dtype=torch.int32, device="cuda")
    parent = torch.empty((64, V), dtype=torch.int32, device="cuda")
    gr.bfs_multi(g, srcs, out=(depth, parent))
    m = gr.bfs_multi(g, srcs, out=(depth, parent))[2]
    d1 = torch.empty(V, dtype=torch.int32, device="cuda")
    p1 = torch.empty(V, dtype=torch.int32, device="cuda")
    single_ms = single_teps = 0.0
    for s in srcs:
        st = gr.bfs(g, int(s), opts=ob, out=(d1, p1))[2]
        single_ms += st["device_ms"]
        single_teps += st["teps_edges"]
    out["bfs_64_sources_rmat20"] = {
        "batched_ms": round(m["device_ms"], 3), "batched_gteps": _gteps(m["teps_edges"], m["device_ms"]),
        "single_source_ms": round(single_ms, 3), "single_source_gteps": _gteps(single_teps, single_ms),
        "speedup": round(single_ms / m["device_ms"], 3) if m["device_ms"] > 0 else None}
    del depth, parent
    g.free()
    del hg
    log("# batched bfs done")
    # 256 small graphs, one union SSSP
    parts, psrc = gg.small_rmat_batch(256)
    u, voff = gg.disjoint_union(parts)
    g = gr.Graph.from_host(ctx, u, symmetric=True)
    gsrc = (psrc.astype(np.int64) + voff[:-1]).astype(np.int32)
    ou = autotune.tuned_opts(g, "sssp")
    gr.sssp(g, gsrc, opts=ou)
    b = gr.sssp(g, gsrc, opts=ou)[2]
    g.free()
    single_ms = single_teps = 0.0
    for i, p in enumerate(parts):
        gp = gr.Graph.from_host(ctx, p, symmetric=True)
        st = gr.sssp(gp, [int(psrc[i])], opts=autotune.tuned_opts(gp, "sssp"))[2]
        single_ms += st["device_ms"]
        single_teps += st["teps_edges"]
        gp.free()
    out["sssp_256_small_rmat_union"] = {
        "n_vertices": int(u.n_vertices), "n_edges": int(u.n_edges),
        "batched_ms": round(b["device_ms"], 3), "batched_gteps": _gteps(b["teps_edges"], b["device_ms"]),
        "single_graph_ms": round(single_ms, 3), "single_graph_gteps": _gteps(single_teps, single_ms),
        "speedup": round(single_ms / b["device_ms"], 3) if b["device_ms"] > 0 else None}
    log("# batched sssp done")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; the library has no multi-GPU path (got --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1701_01170_amd as gr
    from paper_1701_01170_amd import graphgen as gg
    if args.large:
        large(args, gr, gg, torch)
        return

    t0 = time.time()
    hg = gg.add_weights(gg.rmat(args.scale, args.edge_factor, seed=1), seed=101)
    srcs = gg.sources(hg, args.steps + args.warmup, seed=1000)
    print(f"# generated {hg.name}: V={hg.n_vertices} E={hg.n_edges} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    ctx = gr.Context(0)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    dev = torch.device("cuda", 0)
    V = hg.n_vertices
    depth = torch.empty(V, dtype=torch.int32, device=dev)
    parent = torch.empty(V, dtype=torch.int32, device=dev)
    dist = torch.empty(V, dtype=torch.int32, device=dev)
    pred = torch.empty(V, dtype=torch.int32, device=dev)
    cap = 4096
    from paper_1701_01170_amd import autotune
    ob, os_, tb, ts = headline_opts(gr, g, cap)
    knobs = {k: {"bfs": getattr(ob, k), "sssp": getattr(os_, k)} for k in autotune.KNOBS}
    stream = torch.cuda.current_stream()

    def step(s):
        _, _, sb = gr.bfs(g, int(s), opts=ob, out=(depth, parent), stream=stream)
        _, _, ss = gr.sssp(g, [int(s)], opts=os_, out=(dist, pred), stream=stream)
        return sb, ss

    for i in range(args.warmup):
        step(srcs[i])
    torch.cuda.synchronize()
    per_kernel = {}  # (kind, kernel) -> [launches, sum_us, sum_bytes]
    teps = bfs_teps = sssp_teps = 0
    bfs_ms = sssp_ms = 0.0
    t0 = time.perf_counter()
    for i in range(args.steps):
        sb, ss = step(srcs[args.warmup + i])
        teps += sb["teps_edges"] + ss["teps_edges"]
        bfs_teps += sb["teps_edges"]
        sssp_teps += ss["teps_edges"]
        bfs_ms += sb["device_ms"]
        sssp_ms += ss["device_ms"]
        for kind, buf, o in (("bfs", tb, ob), ("sssp", ts, os_)):
            for t in buf[:min(o.trace_count, cap)]:
                a = per_kernel.setdefault((kind, t.kernel), [0, 0.0, 0.0])
                a[0] += 1
                a[1] += t.kernel_us
                b = algorithmic_bytes(kind, t.kernel, t.n_f, t.m_f, t.n_next)
                a[2] += b if b is not None else float("nan")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = teps / wall / 1e9

    # the same steps with the paper's default knobs, for comparison (untimed by the step clock)
    paper_ms = {"bfs": 0.0, "sssp": 0.0}
    for i in range(args.steps):
        s = int(srcs[args.warmup + i])
        paper_ms["bfs"] += gr.bfs(g, s, out=(depth, parent), stream=stream)[2]["device_ms"]
        paper_ms["sssp"] += gr.sssp(g, [s], out=(dist, pred), stream=stream)[2]["device_ms"]

    # the learned selector on the same sources (when trained weights exist)
    learned = None
    from paper_1701_01170_amd import selector
    if not args.no_extras and os.path.exists(selector.WEIGHTS):
        ctx.set_policy(np.load(selector.WEIGHTS))
        # the network picks each iteration's action; thresholds and chunk
        # sizes are the same tuned values as the headline run's
        olb = autotune.tuned_opts(g, "bfs", policy=gr.POLICY_LEARNED)
        ols = autotune.tuned_opts(g, "sssp", policy=gr.POLICY_LEARNED)
        lm = {"bfs": 0.0, "sssp": 0.0}
        for i in range(args.steps):
            s = int(srcs[args.warmup + i])
            lm["bfs"] += gr.bfs(g, s, opts=olb, out=(depth, parent), stream=stream)[2]["device_ms"]
            lm["sssp"] += gr.sssp(g, [s], opts=ols, out=(dist, pred), stream=stream)[2]["device_ms"]
        ctx.set_policy(None)
        learned = {"bfs_ms": round(lm["bfs"] / args.steps, 4), "sssp_ms": round(lm["sssp"] / args.steps, 4),
                   "bfs_gteps_device": _gteps(bfs_teps, lm["bfs"]),
                   "sssp_gteps_device": _gteps(sssp_teps, lm["sssp"]),
                   "step_gteps_device": _gteps(bfs_teps + sssp_teps, lm["bfs"] + lm["sssp"]),
                   "heuristic_step_gteps_device": _gteps(bfs_teps + sssp_teps, bfs_ms + sssp_ms)}

    dom = max(per_kernel, key=lambda k: per_kernel[k][1])
    launches, sum_us, sum_bytes = per_kernel[dom]
    achieved = sum_bytes / (sum_us * 1e-6) / 1e9 if sum_us > 0 else None
    copy_gbs = gr.copy_bandwidth(ctx, 1 << 30, 20)
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{KERNEL_NAMES[dom].split('<')[0]}_{dom[0]}_rmat{args.scale}.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("kernel_source_hash") == kernel_source_hash():
            traffic = tj.get("hbm_bytes_per_launch")

    out = {
        "metric": "GTEPS BFS/SSSP RMAT-22, learned+batched vs plain; % HBM peak",
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"rmat_s{args.scale}_e{args.edge_factor} BFS+SSSP from one seeded source "
                               f"per step, fixed-threshold heuristic policy with autotuned thresholds, "
                               f"int32 CSR, uint32 weights 1..64",
                   "n_vertices": V, "n_edges": hg.n_edges,
                   "knobs": {k: {t: round(float(x), 6) for t, x in v.items()} for k, v in knobs.items()}},
        "roofline": {
            "bound": "hbm",
            "kernel": KERNEL_NAMES[dom],
            "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launches": launches,
            "avg_launch_us": round(sum_us / launches, 2),
            "algorithmic_bytes_per_launch": round(sum_bytes / launches),
            "copy_ceiling_gbs": round(copy_gbs, 1),
        },
        "breakdown": {
            "bfs_gteps_device": round(bfs_teps / (bfs_ms / 1e3) / 1e9, 3),
            "sssp_gteps_device": round(sssp_teps / (sssp_ms / 1e3) / 1e9, 3),
            "bfs_ms": round(bfs_ms / args.steps, 4),
            "sssp_ms": round(sssp_ms / args.steps, 4),
            "paper_default_knobs_bfs_ms": round(paper_ms["bfs"] / args.steps, 4),
            "paper_default_knobs_sssp_ms": round(paper_ms["sssp"] / args.steps, 4),
            "kernel_us_per_step": {f"{k[0]}:{KERNEL_NAMES[k]}": round(v[1] / args.steps, 1)
                                   for k, v in sorted(per_kernel.items())},
        },
        "cpu_baseline": None,
    }

    out["breakdown"]["learned_selector"] = learned
    if not args.no_extras:
        out["breakdown"].update(extras(gr, gg, ctx, torch,
                                       lambda m: print(m, file=sys.stderr, flush=True)))

    if not args.no_cpu_baseline:
        import oracle
        # BFS + SSSP pairs from the step's sources until about 10 s of CPU work
        t_b = t_s = 0.0
        te = 0
        used = []
        for k in range(4):
            s0 = int(srcs[(args.warmup + k) % len(srcs)])
            t0 = time.perf_counter()
            d, _ = oracle.bfs(hg.row_offsets, hg.col_indices, s0)
            t_b += time.perf_counter() - t0
            t0 = time.perf_counter()
            dd, _ = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s0])
            t_s += time.perf_counter() - t0
            te += oracle.teps_edges(hg.row_offsets, d >= 0) + oracle.teps_edges(hg.row_offsets, dd != 0xFFFFFFFF)
            used.append(s0)
            if t_b + t_s >= 10.0:
                break
        out["cpu_baseline"] = {"value": round(te / (t_b + t_s) / 1e9, 6), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{len(used)} BFS + SSSP pairs (each with its parent/predecessor "
                                         f"pass) from sources {used} of the same graph: bfs {t_b:.2f}s, "
                                         f"sssp {t_s:.2f}s in total, single thread"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
