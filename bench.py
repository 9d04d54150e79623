"""Benchmark: BFS and SSSP on an undirected R-MAT graph of scale 22 (edge
factor 16, a=0.57 b=0.19 c=0.19 d=0.05, uint32 weights uniform in 1..64),
on one MI355X.

A step is one pass of the traversal hot path over the resident graph: a
direction-optimising BFS (depths + canonical parents) and an SSSP (distances +
canonical predecessors) from the same seeded source, each selecting its
advance strategy per iteration with the fixed-threshold heuristic.  The graph
is generated on the host and uploaded before the timed region.  Throughput is
GTEPS = (sum over the step's traversals of the degrees of reached vertices) /
step time, the paper's TEPS convention (Sec. 7, measurement methodology).

Prints ONE JSON line (see --help).  The CPU oracle (single thread) is timed
on a bounded sample of the same workload as `cpu_baseline`.
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

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1701_01170_amd as gr
    from paper_1701_01170_amd import graphgen as gg

    t0 = time.time()
    hg = gg.add_weights(gg.rmat(args.scale, args.edge_factor, seed=1), seed=101)
    srcs = gg.sources(hg, args.steps + args.warmup, seed=1000)
    gen_s = time.time() - t0
    print(f"# generated {hg.name}: V={hg.n_vertices} E={hg.n_edges} in {gen_s:.1f}s", file=sys.stderr,
          flush=True)

    ctx = gr.Context(0)
    g = gr.Graph.from_host(ctx, hg, symmetric=True)
    dev = torch.device("cuda", 0)
    V = hg.n_vertices
    depth = torch.empty(V, dtype=torch.int32, device=dev)
    parent = torch.empty(V, dtype=torch.int32, device=dev)
    dist = torch.empty(V, dtype=torch.int32, device=dev)
    pred = torch.empty(V, dtype=torch.int32, device=dev)
    opts = gr.default_opts()

    def step(s):
        _, _, sb = gr.bfs(g, int(s), opts=opts, out=(depth, parent))
        _, _, ss = gr.sssp(g, [int(s)], opts=opts, out=(dist, pred))
        return sb, ss

    for i in range(args.warmup):
        step(srcs[i])
    torch.cuda.synchronize()
    teps = 0
    bfs_ms = sssp_ms = 0.0
    bfs_teps = sssp_teps = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        sb, ss = step(srcs[args.warmup + i])
        teps += sb["teps_edges"] + ss["teps_edges"]
        bfs_teps += sb["teps_edges"]
        sssp_teps += ss["teps_edges"]
        bfs_ms += sb["device_ms"]
        sssp_ms += ss["device_ms"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = teps / wall / 1e9

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
        "config": {"workload": f"rmat_s{args.scale}_e{args.edge_factor} BFS+SSSP single source, heuristic",
                   "n_vertices": V, "n_edges": hg.n_edges, "sources_per_step": 1},
        "breakdown": {
            "bfs_gteps_device": round(bfs_teps / (bfs_ms / 1e3) / 1e9, 3),
            "sssp_gteps_device": round(sssp_teps / (sssp_ms / 1e3) / 1e9, 3),
            "bfs_ms": round(bfs_ms / args.steps, 4),
            "sssp_ms": round(sssp_ms / args.steps, 4),
        },
        "roofline": None,
        "cpu_baseline": None,
    }

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        s0 = int(srcs[args.warmup])
        d, _ = oracle.bfs(hg.row_offsets, hg.col_indices, s0)
        t_b = time.perf_counter() - t0
        t0 = time.perf_counter()
        dd, _ = oracle.sssp(hg.row_offsets, hg.col_indices, hg.weights, [s0])
        t_s = time.perf_counter() - t0
        te = oracle.teps_edges(hg.row_offsets, d >= 0) + oracle.teps_edges(hg.row_offsets, dd != 0xFFFFFFFF)
        out["cpu_baseline"] = {"value": round(te / (t_b + t_s) / 1e9, 6), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one BFS + one SSSP (with parent/pred passes) from source {s0}, "
                                         f"bfs {t_b:.2f}s sssp {t_s:.2f}s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
