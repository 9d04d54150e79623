"""Benchmark: BFS and SSSP on an undirected R-MAT graph of scale 22 (edge
factor 16, a=0.57 b=0.19 c=0.19 d=0.05, uint32 weights uniform in 1..64),
on one MI355X.

A step is one pass of the traversal hot path over the resident graph: a
direction-optimising BFS (depths + canonical parents) and an SSSP (distances +
canonical predecessors) from the same seeded source, each choosing its advance
strategy per iteration with the fixed-threshold heuristic of the paper, its
knobs set by the autotuner.  The graph is generated on the host and uploaded
before the timed region.  Throughput is GTEPS = (sum over the step's
traversals of the degrees of the reached vertices) / step time, the paper's
TEPS convention (Sec. 7, measurement methodology).

The timed steps run with per-iteration tracing on, so every advance kernel is
bracketed by HIP events on the traversal's stream.  `roofline` divides the
algorithmic bytes of the dominant advance kernel by its event-timed duration;
`roofline_bfs` does the same for the BFS alone (its dominant kernel, and the
whole BFS over its device time).  `traffic` comes from committed rocprofv3
FETCH_SIZE/WRITE_SIZE summaries (profiles/traffic_*.json) when they were
taken on the current kernel source, else null; those counters measure the
bytes between the L2 caches and the memory fabric (Infinity Cache hits
included), an upper bound of HBM bytes.  `cpu_baseline` times the CPU oracle
(single thread) on BFS + SSSP pairs of the same workload (about 10 s of CPU
work).

Side by side (breakdown): the learned selector against the heuristic, both
untraced, interleaved per source; the R-MAT scale 14 BFS (single source, and
learned against heuristic; degree-renumbered, with the generation-order time
beside it); the 2048 x 2048 grid; batched BFS (R-MAT 20, renumbered and in
generation order) and the 256-graph union SSSP against single runs;
betweenness centrality on the headline graph; the BFS filter x direction
optimisation ablation.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
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
    ("bfs", 11): "k_bfs_pull_list",
}


def algorithmic_bytes(kind: str, kernel: int, n_f: int, m_f: int, n_next: int, n_in: int = 0,
                      inspected: int = 0, V: int = 0) -> float:
    """Bytes the method must move for one advance launch (trace record fields):
    SSSP relax: per edge 4 B column + 4 B weight + 8 B packed atomic-min of the
      target's (dist, pred) key; per frontier vertex 4 B id + 8 B row offsets;
      per output vertex 4 B queue entry.
    SSSP priority-queue refill: per far-pile entry 4 B id + 8 B key + 4 B
      written to the next frontier or the next far pile.
    BFS push: per edge 4 B column (the visited test is one bit, cache
      resident); per frontier vertex 12 B; per new vertex 4 B depth + 4 B
      parent + 4 B queue entry.
    BFS pull over the bitmap: the visited bitmap once (V / 4 B: two words per
      32 vertices), 8 B row offsets per unvisited vertex, 4 B per neighbour
      scanned (its frontier bit is cache resident), 12 B per vertex found.
    BFS pull over the unvisited list: 4 B entry + 8 B row offsets per list
      entry, 4 B per neighbour scanned, 12 B per vertex found."""
    if kind == "sssp":
        if kernel == 7:
            return 16.0 * n_in
        return 16.0 * m_f + 12.0 * n_f + 4.0 * n_next
    if kernel in (4, 5):
        return V / 4.0 + 8.0 * n_in + 4.0 * inspected + 12.0 * n_next
    if kernel == 11:
        return 12.0 * n_in + 4.0 * inspected + 12.0 * n_next
    return 4.0 * m_f + 12.0 * n_f + 12.0 * n_next


def accumulate(per_kernel: dict, kind: str, buf, count: int, V: int) -> float:
    """Adds one traversal's trace records to per_kernel[(kind, kernel)] =
    [launches, sum of event-timed us, sum of algorithmic bytes]; returns the
    traversal's total algorithmic bytes."""
    total = 0.0
    for t in buf[:count]:
        a = per_kernel.setdefault((kind, t.kernel), [0, 0.0, 0.0])
        b = algorithmic_bytes(kind, t.kernel, t.n_f, t.m_f, t.n_next, t.n_in, t.inspected, V)
        a[0] += 1
        a[1] += t.kernel_us
        a[2] += b
        total += b
    return total


def roofline_of(per_kernel: dict, key) -> dict:
    launches, sum_us, sum_bytes = per_kernel[key]
    achieved = sum_bytes / (sum_us * 1e-6) / 1e9 if sum_us > 0 else None
    return {"bound": "hbm", "kernel": KERNEL_NAMES[key],
            "achieved": None if achieved is None else round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "launches": launches, "avg_launch_us": round(sum_us / launches, 2),
            "algorithmic_bytes_per_launch": round(sum_bytes / launches)}


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": aff}


def headline_opts(gr, g, cap: int = 4096):
    """The timed configuration of the headline step: the heuristic policy with
    the knobs the autotuner stored for this graph's class and size (paper
    defaults when none are stored), and per-iteration tracing into host
    buffers of `cap` records (advance kernels only: trace_steps_off).
    Returns (bfs opts, sssp opts, bfs trace, sssp trace); the trace buffers
    must outlive the opts."""
    from paper_1701_01170_amd import autotune
    tb = (gr.LevelTrace * cap)()
    ts = (gr.LevelTrace * cap)()
    ob = autotune.tuned_opts(g, "bfs", trace=tb, trace_capacity=cap, trace_steps_off=1)
    os_ = autotune.tuned_opts(g, "sssp", trace=ts, trace_capacity=cap, trace_steps_off=1)
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
                    help="skip the side-by-side comparisons (learned, R-MAT 14, grid, batched)")
    ap.add_argument("--large", action="store_true",
                    help="instead of the headline, run the largest workload: R-MAT scale 25, "
                         "16-source batched BFS and 16 SSSP runs")
    return ap.parse_args()


def _gteps(teps: float, ms: float) -> float | None:
    return round(teps / (ms * 1e-3) / 1e9, 3) if ms > 0 else None


def _fabric_traffic(dom, scale: int) -> tuple[float | None, dict | None]:
    """The committed counter summary of the dominant kernel, if it was taken
    on the current kernel source: (scaled L2 <-> fabric bytes per launch,
    the summary's fields)."""
    tfile = os.path.join(ROOT, "profiles",
                         f"traffic_{KERNEL_NAMES[dom].split('<')[0]}_{dom[0]}_rmat{scale}.json")
    if not os.path.exists(tfile):
        return None, None
    with open(tfile) as fh:
        tj = json.load(fh)
    if tj.get("kernel_source_hash") != kernel_source_hash():
        return None, {"stale": os.path.relpath(tfile, ROOT)}
    return tj.get("l2_fabric_bytes_per_launch"), {
        "file": os.path.relpath(tfile, ROOT), "unscaled_bytes_per_launch": tj.get("unscaled_bytes_per_launch"),
        "meaning": tj.get("meaning")}


def compare_policies(gr, g, sources, opts_a, opts_b, kinds=("bfs", "sssp"), outs=None):
    """Device time of two option sets on the same sources, both untraced,
    interleaved (a then b on even sources, b then a on odd ones).  Returns
    {kind: {"a_ms": [...], "b_ms": [...], "teps": [...]}}."""
    res = {k: {"a_ms": [], "b_ms": [], "teps": []} for k in kinds}
    for i, s in enumerate(sources):
        for kind in kinds:
            order = (("a", opts_a[kind]), ("b", opts_b[kind]))
            if i % 2:
                order = order[::-1]
            for label, o in order:
                out = None if outs is None else outs[kind]
                if kind == "bfs":
                    st = gr.bfs(g, int(s), opts=o, out=out)[2]
                else:
                    st = gr.sssp(g, [int(s)], opts=o, out=out)[2]
                res[kind][label + "_ms"].append(st["device_ms"])
            res[kind]["teps"].append(st["teps_edges"])
    return res


def summarize_pair(res: dict, a_name: str, b_name: str) -> dict:
    """Medians, sums and the spread of the per-source time ratio b / a."""
    out = {}
    tot_a = tot_b = tot_t = 0.0
    for kind, r in res.items():
        ratio = [b / a for a, b in zip(r["a_ms"], r["b_ms"]) if a > 0]
        out[kind] = {f"{a_name}_median_ms": round(statistics.median(r["a_ms"]), 4),
                     f"{b_name}_median_ms": round(statistics.median(r["b_ms"]), 4),
                     f"{a_name}_gteps": _gteps(sum(r["teps"]), sum(r["a_ms"])),
                     f"{b_name}_gteps": _gteps(sum(r["teps"]), sum(r["b_ms"])),
                     f"time_ratio_{b_name}_over_{a_name}": {
                         "median": round(statistics.median(ratio), 4), "min": round(min(ratio), 4),
                         "max": round(max(ratio), 4)}}
        tot_a += sum(r["a_ms"])
        tot_b += sum(r["b_ms"])
        tot_t += sum(r["teps"])
    out["sources"] = len(next(iter(res.values()))["a_ms"])
    out[f"step_{a_name}_gteps"] = _gteps(tot_t, tot_a)
    out[f"step_{b_name}_gteps"] = _gteps(tot_t, tot_b)
    out[f"step_{b_name}_speedup"] = round(tot_a / tot_b, 4) if tot_b > 0 else None
    return out


def learned_vs_heuristic(gr, g, ctx, sources, outs=None) -> dict | None:
    """The trained selector against the tuned heuristic, same knobs, both
    untraced, interleaved per source (None without trained weights)."""
    from paper_1701_01170_amd import autotune, selector
    if not os.path.exists(selector.WEIGHTS):
        return None
    selector.load_policy(ctx)
    oh = {k: autotune.tuned_opts(g, k) for k in ("bfs", "sssp")}
    ol = {k: autotune.tuned_opts(g, k, policy=gr.POLICY_LEARNED) for k in ("bfs", "sssp")}
    res = compare_policies(gr, g, sources, oh, ol, outs=outs)
    ctx.set_policy(None)
    return summarize_pair(res, "heuristic", "learned")


def filter_ablation(gr, g, sources, outs) -> dict:
    """BFS under the paper's idempotence x direction-optimisation ablation
    (Sec. 7, optimisation analysis): the filter of the push levels (auto:
    atomic culling on small levels, atomic-free byte marks on large ones;
    atomic: the first atomic OR of a vertex's visited bit appends it on every
    level, the LB_CULL-style exact filter; idempotent: no atomics in the
    advance, inexact culling heuristics, then an exact filter pass) with and
    without the push -> pull switch.  Tuned knobs otherwise, untraced, the
    variants interleaved per source.  A traced run per variant gives the
    duplicates the idempotent heuristics let through (candidates / exact new
    vertices over its idempotent levels)."""
    import math
    from paper_1701_01170_amd import autotune
    variants = {}
    for fname, fv in (("auto", gr.BFS_FILTER_AUTO), ("atomic", gr.BFS_FILTER_ATOMIC),
                      ("idempotent", gr.BFS_FILTER_IDEMPOTENT)):
        for dname, do_kw in (("do", {}), ("no_do", {"do_a": math.inf})):
            variants[f"{fname}_{dname}"] = autotune.tuned_opts(g, "bfs", bfs_filter=fv, **do_kw)
    ms = {k: [] for k in variants}
    teps = []
    for i, s in enumerate(sources):
        names = list(variants)
        if i % 2:
            names = names[::-1]
        for k in names:
            st = gr.bfs(g, int(s), opts=variants[k], out=outs)[2]
            ms[k].append(st["device_ms"])
        teps.append(st["teps_edges"])
    out = {"sources": len(sources)}
    base = sum(ms["auto_do"])
    for k in variants:
        out[k] = {"median_ms": round(statistics.median(ms[k]), 4),
                  "gteps": _gteps(sum(teps), sum(ms[k])),
                  "time_over_auto_do": round(sum(ms[k]) / base, 4) if base > 0 else None}
    cap = 512
    for k in ("idempotent_do", "idempotent_no_do"):
        tr = (gr.LevelTrace * cap)()
        o = autotune.tuned_opts(g, "bfs", bfs_filter=variants[k].bfs_filter, do_a=variants[k].do_a,
                                trace=tr, trace_capacity=cap)
        cand = exact = 0
        for s in sources[:4]:
            gr.bfs(g, int(s), opts=o, out=outs)
            for r in tr[:min(o.trace_count, cap)]:
                if r.kernel >= 12:
                    cand += r.n_cand
                    exact += r.n_next
        out[k]["candidates_over_new_vertices"] = round(cand / exact, 4) if exact else None
    return out


def rmat14(gr, gg, ctx) -> dict:
    """R-MAT scale 14: the single-source BFS (median device us and GTEPS over
    20 seeded sources, tuned heuristic, untraced) and the learned selector
    against the heuristic on the same graph (BFS and SSSP)."""
    from paper_1701_01170_amd import autotune
    hg = gg.add_weights(gg.rmat(14, 16, seed=1), seed=101)
    # degree-renumbered ingest, the layout the tuner and the selector's
    # training traces use (results in the caller's ids)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    srcs = gg.sources(hg, 20, seed=1000)
    ob = autotune.tuned_opts(g, "bfs")
    gr.bfs(g, int(srcs[0]), opts=ob)
    ms, te = [], []
    for s in srcs:
        st = gr.bfs(g, int(s), opts=ob)[2]
        ms.append(st["device_ms"])
        te.append(st["teps_edges"])
    out = {"graph": f"rmat_s14_e16 (V={hg.n_vertices}, E={hg.n_edges}), degree-renumbered ingest",
           "bfs_median_us": round(1e3 * statistics.median(ms), 2),
           "bfs_min_us": round(1e3 * min(ms), 2), "bfs_max_us": round(1e3 * max(ms), 2),
           "bfs_gteps": _gteps(sum(te), sum(ms)), "sources": len(srcs)}
    # iteration control: per-level cost with device blocks (enqueued, or
    # recorded as hipGraphs) and with a host round trip per level
    levels = {}
    for label, kw in (("device_blocks", {}), ("device_blocks_graph", {"graph_blocks": 1}),
                      ("host_loop", {"device_max_edges": -1})):
        o = autotune.tuned_opts(g, "bfs", **kw)
        gr.bfs(g, int(srcs[0]), opts=o)
        tot_ms = tot_it = 0
        for s in srcs:
            st = gr.bfs(g, int(s), opts=o)[2]
            tot_ms += st["device_ms"]
            tot_it += st["iterations"]
        levels[label] = {"us_per_level": round(1e3 * tot_ms / max(1, tot_it), 2),
                         "bfs_mean_us": round(1e3 * tot_ms / len(srcs), 2)}
    out["iteration_control"] = levels
    out["learned_vs_heuristic"] = learned_vs_heuristic(gr, g, ctx, gg.sources(hg, 20, seed=1100))
    g.free()
    # the same BFS on the graph in generation order (no renumbering), which
    # is faster at this size
    g0 = gr.Graph.from_host(ctx, hg, symmetric=True)
    gr.bfs(g0, int(srcs[0]), opts=ob)
    ms0, te0 = [], []
    for s in srcs:
        st = gr.bfs(g0, int(s), opts=ob)[2]
        ms0.append(st["device_ms"])
        te0.append(st["teps_edges"])
    out["generation_order"] = {"bfs_median_us": round(1e3 * statistics.median(ms0), 2),
                               "bfs_gteps": _gteps(sum(te0), sum(ms0))}
    g0.free()
    return out


def extras(gr, gg, ctx, torch, log):
    """Comparison workloads reported next to the headline (device-event time):
    the 2048 x 2048 grid (high diameter, small frontiers), 64-source batched BFS
    on R-MAT scale 20 against 64 single-source runs, 256 small R-MAT graphs in
    one disjoint-union SSSP against 256 separate runs."""
    from paper_1701_01170_amd import autotune
    out = {}
    # grid
    hg = gg.add_weights(gg.grid(2048, 2048), seed=101)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    s = int(gg.sources(hg, 1, seed=1000)[0])
    row = {}
    for label, kw in (("device_blocks", {}), ("device_blocks_graph", {"graph_blocks": 1}),
                      ("host_loop", {"device_max_edges": -1})):
        ob = autotune.tuned_opts(g, "bfs", **kw)
        os_ = autotune.tuned_opts(g, "sssp", **kw)
        gr.bfs(g, s, opts=ob)
        b = gr.bfs(g, s, opts=ob)[2]
        t = gr.sssp(g, [s], opts=os_)[2]
        row[label] = {"bfs_ms": round(b["device_ms"], 3), "bfs_gteps": _gteps(b["teps_edges"], b["device_ms"]),
                      "bfs_iterations": b["iterations"],
                      "bfs_us_per_level": round(1e3 * b["device_ms"] / max(1, b["iterations"]), 2),
                      "sssp_ms": round(t["device_ms"], 3),
                      "sssp_gteps": _gteps(t["teps_edges"], t["device_ms"]), "sssp_iterations": t["iterations"],
                      "sssp_us_per_level": round(1e3 * t["device_ms"] / max(1, t["iterations"]), 2)}
    out["grid_2048x2048"] = row
    g.free()
    del hg
    log("# grid done")
    # 64-source batched BFS, R-MAT scale 20
    hg = gg.rmat(20, 16, seed=1)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    srcs = gg.sources(hg, 64, seed=2000).astype(np.int32)
    ob = autotune.tuned_opts(g, "bfs")
    om = autotune.tuned_opts(g, "bfs_multi")
    V = hg.n_vertices
    depth = torch.empty((64, V), dtype=torch.int32, device="cuda")
    parent = torch.empty((64, V), dtype=torch.int32, device="cuda")
    gr.bfs_multi(g, srcs, opts=om, out=(depth, parent))
    m = gr.bfs_multi(g, srcs, opts=om, out=(depth, parent))[2]
    d1 = torch.empty(V, dtype=torch.int32, device="cuda")
    p1 = torch.empty(V, dtype=torch.int32, device="cuda")
    single_ms = single_teps = 0.0
    for s in srcs:
        st = gr.bfs(g, int(s), opts=ob, out=(d1, p1))[2]
        single_ms += st["device_ms"]
        single_teps += st["teps_edges"]
    out["bfs_64_sources_rmat20"] = {
        "graph": "rmat_s20_e16, degree-renumbered ingest",
        "batched_ms": round(m["device_ms"], 3), "batched_gteps": _gteps(m["teps_edges"], m["device_ms"]),
        "batched_iterations": m["iterations"],
        "single_source_ms": round(single_ms, 3), "single_source_gteps": _gteps(single_teps, single_ms),
        "speedup": round(single_ms / m["device_ms"], 3) if m["device_ms"] > 0 else None}
    # the batched network against the heuristic: five 64-source batches each,
    # interleaved, same tuned knobs
    from paper_1701_01170_amd import selector
    if selector.load_policy(ctx):
        ol = autotune.tuned_opts(g, "bfs_multi", policy=gr.POLICY_LEARNED)
        hm, lm, te = [], [], []
        for b in range(5):
            sb = gg.sources(hg, 64, seed=2300 + b).astype(np.int32)
            pair = [("h", om), ("l", ol)] if b % 2 == 0 else [("l", ol), ("h", om)]
            for label, o in pair:
                st = gr.bfs_multi(g, sb, opts=o, out=(depth, parent))[2]
                (hm if label == "h" else lm).append(st["device_ms"])
            te.append(st["teps_edges"])
        ctx.set_policy(None)
        out["bfs_64_sources_rmat20"]["learned_vs_heuristic"] = {
            "batches": 5, "heuristic_median_ms": round(statistics.median(hm), 4),
            "learned_median_ms": round(statistics.median(lm), 4),
            "heuristic_gteps": _gteps(sum(te), sum(hm)), "learned_gteps": _gteps(sum(te), sum(lm)),
            "learned_speedup": round(sum(hm) / sum(lm), 4) if sum(lm) > 0 else None}
    g.free()
    # the batched and the single-source runs on the graph in generation order
    g0 = gr.Graph.from_host(ctx, hg, symmetric=True)
    gr.bfs_multi(g0, srcs, opts=om, out=(depth, parent))
    m0 = gr.bfs_multi(g0, srcs, opts=om, out=(depth, parent))[2]
    single0 = 0.0
    for s in srcs:
        single0 += gr.bfs(g0, int(s), opts=ob, out=(d1, p1))[2]["device_ms"]
    out["bfs_64_sources_rmat20"]["generation_order"] = {
        "batched_ms": round(m0["device_ms"], 3), "single_source_ms": round(single0, 3),
        "speedup": round(single0 / m0["device_ms"], 3) if m0["device_ms"] > 0 else None}
    g0.free()
    del depth, parent
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


def bc_rmat22(gr, g, sources) -> dict:
    """Betweenness centrality (gr_bc, Brandes's two passes on the advance
    operator) from each source alone and from all of them in one call: device
    time and the rate over the reached vertices' edges per source (teps_edges
    of the stats; each pass then sweeps, per pair of adjacent levels, the rows
    of one of the two), with the autotuner's knobs for BC."""
    from paper_1701_01170_amd import autotune
    o = autotune.tuned_opts(g, "bc")
    gr.bc(g, [int(sources[0])], opts=o)  # warm-up
    ms, te = [], 0
    for s in sources:
        st = gr.bc(g, [int(s)], opts=o)[2]
        ms.append(st["device_ms"])
        te += st["teps_edges"]
    allst = gr.bc(g, [int(s) for s in sources], opts=o)[2]
    # the per-pair choice against each form alone (same knobs and sources)
    forms = {}
    for name, dirs in (("push_both", gr.BC_DIR_PUSH | gr.BC_DIR_PUSH << 2),
                       ("pull_both", gr.BC_DIR_PULL | gr.BC_DIR_PULL << 2)):
        of = autotune.tuned_opts(g, "bc", bc_dir=dirs)
        fm = [gr.bc(g, [int(s)], opts=of)[2]["device_ms"] for s in sources]
        forms[name] = round(statistics.median(fm), 4)
    return {"sources": len(sources), "knobs": {"lb_chunk": o.lb_chunk, "adv_block": o.adv_block},
            "median_ms_per_source": round(statistics.median(ms), 4),
            "gteps": _gteps(te, sum(ms)),
            "all_sources_one_call_ms": round(allst["device_ms"], 4),
            "all_sources_one_call_gteps": _gteps(allst["teps_edges"], allst["device_ms"]),
            "median_ms_per_source_by_form": forms}


def cpu_baseline(hg, srcs, budget_s: float = 10.0, max_pairs: int = 4) -> dict:
    """The CPU oracle (single thread) on BFS + SSSP pairs of the same graph,
    until about budget_s seconds of CPU work."""
    import oracle
    t_b = t_s = 0.0
    te = 0
    used = []
    for s0 in srcs[:max_pairs]:
        s0 = int(s0)
        t0 = time.perf_counter()
        d, _ = oracle.bfs(hg.row_offsets, hg.col_indices, s0)
        t_b += time.perf_counter() - t0
        t0 = time.perf_counter()
        dd, _ = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s0])
        t_s += time.perf_counter() - t0
        te += oracle.teps_edges(hg.row_offsets, d >= 0) + oracle.teps_edges(hg.row_offsets, dd != 0xFFFFFFFF)
        used.append(s0)
        if t_b + t_s >= budget_s:
            break
    hi = host_info()
    return {"value": round(te / (t_b + t_s) / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{len(used)} BFS + SSSP pairs (each with its parent/predecessor pass) from "
                      f"sources {used} of the same graph: bfs {t_b:.2f}s, sssp {t_s:.2f}s in total, "
                      f"single thread",
            "host": hi}


def large(args, gr, gg, torch):
    """R-MAT scale 25 (edge factor 16, ~1.07B directed edges, uint32 weights
    1..64) resident in HBM: one 16-source batched BFS and one 16-source batched
    SSSP (gr_sssp_multi) are the timed step.  Next to them, for comparison, 16
    single-source SSSP runs back to back under the learned selector when
    trained weights exist (else the heuristic); those runs are traced, so the
    single-source relaxation kernel gets a roofline and an achieved GB/s.
    Prints its own JSON line."""
    from paper_1701_01170_amd import autotune, selector
    t0 = time.time()
    hg = gg.add_weights(gg.rmat(25, 16, seed=1), seed=101)
    print(f"# generated {hg.name}: V={hg.n_vertices} E={hg.n_edges} in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ctx = gr.Context(0)
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
    srcs = gg.sources(hg, 16, seed=1000).astype(np.int32)
    V = hg.n_vertices
    policy = "learned" if selector.load_policy(ctx) else "heuristic"
    kw = {"policy": gr.POLICY_LEARNED} if policy == "learned" else {}
    depth = torch.empty((16, V), dtype=torch.int32, device="cuda")
    parent = torch.empty((16, V), dtype=torch.int32, device="cuda")
    om = autotune.tuned_opts(g, "bfs_multi", **kw)
    gr.bfs_multi(g, srcs[:2], opts=om, out=(depth[:2], parent[:2]))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mb = gr.bfs_multi(g, srcs, opts=om, out=(depth, parent))[2]
    torch.cuda.synchronize()
    bfs_wall = time.perf_counter() - t0
    # the same batch under the heuristic, for comparison (untimed by the step clock)
    mbh = gr.bfs_multi(g, srcs, opts=autotune.tuned_opts(g, "bfs_multi"), out=(depth, parent))[2]
    del depth, parent
    # batched SSSP: the 16 sources in one sweep per iteration
    dist16 = torch.empty((16, V), dtype=torch.int32, device="cuda")
    pred16 = torch.empty((16, V), dtype=torch.int32, device="cuda")
    omsssp = autotune.tuned_opts(g, "sssp_multi")
    gr.sssp_multi(g, srcs[:2], opts=omsssp, out=(dist16[:2], pred16[:2]))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms16 = gr.sssp_multi(g, srcs, opts=omsssp, out=(dist16, pred16))[2]
    torch.cuda.synchronize()
    msssp_wall = time.perf_counter() - t0
    # the other batching mode, for comparison (untimed by the step clock)
    oshared = autotune.tuned_opts(g, "sssp_multi", sssp_multi_sweep=1 - omsssp.sssp_multi_sweep)
    if oshared.sssp_multi_sweep == 0:
        oshared.lb_chunk, oshared.sssp_delta = 0, 0
    ms16_other = gr.sssp_multi(g, srcs, opts=oshared, out=(dist16, pred16))[2]
    del dist16, pred16
    dist = torch.empty(V, dtype=torch.int32, device="cuda")
    pred = torch.empty(V, dtype=torch.int32, device="cuda")
    cap = 4096
    ts = (gr.LevelTrace * cap)()
    os_ = autotune.tuned_opts(g, "sssp", trace=ts, trace_capacity=cap, **kw)
    gr.sssp(g, [int(srcs[0])], opts=os_, out=(dist, pred))
    torch.cuda.synchronize()
    per_kernel = {}
    sssp_bytes = 0.0
    t0 = time.perf_counter()
    steps = []
    for s in srcs:
        steps.append(gr.sssp(g, [int(s)], opts=os_, out=(dist, pred))[2])
        sssp_bytes += accumulate(per_kernel, "sssp", ts, min(os_.trace_count, cap), V)
    torch.cuda.synchronize()
    sssp_wall = time.perf_counter() - t0
    teps = mb["teps_edges"] + ms16["teps_edges"]
    wall = bfs_wall + msssp_wall
    sssp_ms = sum(st["device_ms"] for st in steps)
    serial_teps = mb["teps_edges"] + sum(st["teps_edges"] for st in steps)
    dom = max(per_kernel, key=lambda k: per_kernel[k][1])
    roof = roofline_of(per_kernel, dom)
    roof["traffic"] = None
    out = {
        "metric": "GTEPS BFS/SSSP RMAT-25, 16-source batched BFS + 16-source batched SSSP",
        "value": round(teps / wall / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
        "ms_per_step": round(wall * 1e3, 3), "higher_is_better": True, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "rmat_s25_e16, int32 CSR degree-renumbered on ingest (results in the "
                               "caller's ids), uint32 weights 1..64; gr_bfs_multi with 16 sources + "
                               "gr_sssp_multi with the same 16 sources",
                   "policy": {"sssp_single_source_comparison": policy,
                              "bfs_multi": policy + " (batched network when trained)",
                              "sssp_multi": ("one source per sweep (tuned)" if omsssp.sssp_multi_sweep
                                             else "sources share each sweep (tuned)")},
                   "n_vertices": V, "n_edges": g.n_edges},
        "roofline": roof,
        "breakdown": {"bfs_multi16_ms": round(mb["device_ms"], 3),
                      "bfs_multi16_gteps_device": _gteps(mb["teps_edges"], mb["device_ms"]),
                      "bfs_multi16_heuristic_ms": round(mbh["device_ms"], 3),
                      "sssp_multi16_ms": round(ms16["device_ms"], 3),
                      "sssp_multi16_gteps_device": _gteps(ms16["teps_edges"], ms16["device_ms"]),
                      "sssp_multi16_iterations": ms16["iterations"],
                      "sssp_multi16_knobs": {"lb_chunk": omsssp.lb_chunk,
                                             "sssp_delta": omsssp.sssp_delta,
                                             "sssp_multi_sweep": omsssp.sssp_multi_sweep},
                      "sssp_multi16_other_sweep_mode_ms": round(ms16_other["device_ms"], 3),
                      "sssp_multi16_union_edges": ms16["inspected_edges"],
                      "sssp_batched_speedup_over_16_single": round(sssp_ms / ms16["device_ms"], 3)
                      if ms16["device_ms"] > 0 else None,
                      "step_with_16_single_sssp_gteps": round(serial_teps / (bfs_wall + sssp_wall) / 1e9, 4),
                      "sssp16_ms": round(sssp_ms, 3),
                      "sssp16_gteps_device": _gteps(sum(st["teps_edges"] for st in steps), sssp_ms),
                      "sssp16_algorithmic_gbs": round(sssp_bytes / (sssp_ms * 1e-3) / 1e9, 1),
                      "sssp16_hbm_frac": round(sssp_bytes / (sssp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "kernel_us_per_sssp": {f"{k[0]}:{KERNEL_NAMES[k]}": round(v[1] / len(srcs), 1)
                                             for k, v in sorted(per_kernel.items())}},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # one oracle BFS (~10 s at this size) and no Dijkstra (minutes)
        import oracle
        t0 = time.perf_counter()
        d, _ = oracle.bfs(hg.row_offsets, hg.col_indices, int(srcs[0]))
        tb = time.perf_counter() - t0
        te = oracle.teps_edges(hg.row_offsets, d >= 0)
        out["cpu_baseline"] = {"value": round(te / tb / 1e9, 6), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one BFS with its parent pass from source {int(srcs[0])}: "
                                         f"{tb:.2f}s, single thread",
                               "host": host_info()}
    print(json.dumps(out))


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
    g = gr.Graph.from_host(ctx, hg, symmetric=True, renumber=True)
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
    bfs_bytes = 0.0
    def snapshot(buf, n):
        """A copy of the first n trace records (the per-kernel byte and time
        sums are made after the timed region)."""
        c = (gr.LevelTrace * max(n, 1))()
        ctypes.memmove(c, buf, ctypes.sizeof(gr.LevelTrace) * n)
        return c, n

    traces = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        sb, ss = step(srcs[args.warmup + i])
        teps += sb["teps_edges"] + ss["teps_edges"]
        bfs_teps += sb["teps_edges"]
        sssp_teps += ss["teps_edges"]
        bfs_ms += sb["device_ms"]
        sssp_ms += ss["device_ms"]
        traces.append((snapshot(tb, min(ob.trace_count, cap)), snapshot(ts, min(os_.trace_count, cap))))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = teps / wall / 1e9
    for (cb, nb), (cs, ns) in traces:
        bfs_bytes += accumulate(per_kernel, "bfs", cb, nb, V)
        accumulate(per_kernel, "sssp", cs, ns, V)

    # the same steps with the paper's default knobs, for comparison (untimed by the step clock)
    paper_ms = {"bfs": 0.0, "sssp": 0.0}
    for i in range(args.steps):
        s = int(srcs[args.warmup + i])
        paper_ms["bfs"] += gr.bfs(g, s, out=(depth, parent), stream=stream)[2]["device_ms"]
        paper_ms["sssp"] += gr.sssp(g, [s], out=(dist, pred), stream=stream)[2]["device_ms"]

    dom = max(per_kernel, key=lambda k: per_kernel[k][1])
    roof = roofline_of(per_kernel, dom)
    copy_gbs = gr.copy_bandwidth(ctx, 1 << 30, 20)
    traffic, tinfo = _fabric_traffic(dom, args.scale)
    roof["traffic"] = traffic
    roof["traffic_is"] = ("bytes between the L2 caches and the memory fabric per launch (rocprofv3 "
                          "FETCH_SIZE + WRITE_SIZE, each scaled by its reading for a plain copy kernel); "
                          "Infinity Cache hits count too, so this bounds HBM bytes from above")
    roof["traffic_source"] = tinfo
    if traffic:
        roof["traffic_over_algorithmic"] = round(traffic / roof["algorithmic_bytes_per_launch"], 3)
    roof["limiter"] = ("issue rate and latency of the random 8-byte key gathers (counters: "
                       "profiles/counters_k_push_lb_sssp_rmat22.md)") if dom[0] == "sssp" else None
    roof["copy_ceiling_gbs"] = round(copy_gbs, 1)
    bfs_keys = [k for k in per_kernel if k[0] == "bfs"]
    bdom = max(bfs_keys, key=lambda k: per_kernel[k][1])
    roof_bfs = roofline_of(per_kernel, bdom)
    bfs_gbs = bfs_bytes / (bfs_ms * 1e-3) / 1e9
    roof_bfs["whole_bfs"] = {"algorithmic_bytes_per_bfs": round(bfs_bytes / args.steps),
                             "device_ms_per_bfs": round(bfs_ms / args.steps, 4),
                             "achieved": round(bfs_gbs, 1), "frac": round(bfs_gbs / HBM_PEAK_GBS, 4),
                             "copy_ceiling_frac": round(bfs_gbs / copy_gbs, 4) if copy_gbs else None}

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
                               f"int32 CSR degree-renumbered on ingest (results in the caller's ids), "
                               f"uint32 weights 1..64",
                   "n_vertices": V, "n_edges": hg.n_edges,
                   "knobs": {k: {t: round(float(x), 6) for t, x in v.items()} for k, v in knobs.items()}},
        "roofline": roof,
        "roofline_bfs": roof_bfs,
        "breakdown": {
            "bfs_gteps_device": round(bfs_teps / (bfs_ms / 1e3) / 1e9, 3),
            "sssp_gteps_device": round(sssp_teps / (sssp_ms / 1e3) / 1e9, 3),
            "bfs_ms": round(bfs_ms / args.steps, 4),
            "sssp_ms": round(sssp_ms / args.steps, 4),
            "paper_default_knobs_bfs_ms": round(paper_ms["bfs"] / args.steps, 4),
            "paper_default_knobs_sssp_ms": round(paper_ms["sssp"] / args.steps, 4),
            "kernel_us_per_step": {f"{k[0]}:{KERNEL_NAMES[k]}": round(v[1] / args.steps, 1)
                                   for k, v in sorted(per_kernel.items())},
            "kernel_gbs": {f"{k[0]}:{KERNEL_NAMES[k]}": round(v[2] / (v[1] * 1e-6) / 1e9, 1)
                           for k, v in sorted(per_kernel.items()) if v[1] > 0},
        },
        "cpu_baseline": None,
    }

    if not args.no_extras:
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        # learned against heuristic on the same graph: untraced, interleaved,
        # on held-out sources (not the timed ones)
        out["breakdown"]["learned_vs_heuristic_rmat22"] = learned_vs_heuristic(
            gr, g, ctx, gg.sources(hg, 12, seed=1100),
            outs={"bfs": (depth, parent), "sssp": (dist, pred)})
        log("# learned vs heuristic done")
        out["breakdown"]["bc_rmat22"] = bc_rmat22(gr, g, gg.sources(hg, 4, seed=1300))
        log("# betweenness centrality done")
        out["breakdown"]["bfs_filter_ablation_rmat22"] = filter_ablation(
            gr, g, gg.sources(hg, 8, seed=1200), (depth, parent))
        log("# filter ablation done")
        out["breakdown"]["rmat14"] = rmat14(gr, gg, ctx)
        log("# rmat14 done")
        out["breakdown"].update(extras(gr, gg, ctx, torch, log))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(hg, srcs[args.warmup:])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
