"""Autotuner for the traversal's tuning knobs.

The paper sets its knobs by hand (LB_LIGHT threshold 4096, average degree 5
for LB vs. TWC, Sec. 5.1) and by heat maps over the direction-switch
parameters do_a / do_b (Sec. 7, optimisation analysis).  This module searches
the same knobs on the device it runs on, timing the library's own traversals
(event-timed device time, several seeded sources), and stores the best setting
per (gfx arch, graph class, size bucket, traversal) in `tuning/<arch>.json`.

Search (coordinate descent from the paper's defaults, or from the setting
already stored for the graph's class when that is faster):
  1. lb_light_threshold in {0, 1024, 4096}
  2. lb_chunk in {512, 1024, 2048, 4096, 8192, 16384}
  3. adv_block (workgroup size of the push kernels) in {128, 256, 512}
  4. lb_min_avg_degree in {0 (always LB), 5 (paper), inf (always TWC)}
  5. while TWC is in use: its tier cut-offs, twc_wave_min in {16, 32, 64,
     128, 256} and twc_block_min in {64, ..., 4096} (lists longer than these
     go to a wavefront / the whole workgroup)
  6. SSSP only: sssp_delta in {0 (no priority queue), 8, 16, ..., 256}
  7. BFS / SSSP: device_max_edges in {off, 2^16, 2^18, 2^20} (edge bound of
     the device-predicated level blocks)
  8. BFS only: the do_a x do_b grid {1/2 .. 1/256} x {1/576, 1/64, 1/8},
     then bfs_filter in {auto, atomic, idempotent} (Sec. 5.2)
Batched BFS ("bfs_multi", 64 sources per call) searches 1, 2, 3 and its
push -> pull switch do_a in {1/4 .. 1/64}; batched SSSP ("sssp_multi", 16
sources per call) its chunk {512, 1024, 2048} and sssp_delta {0, 2, ..., 64}
with the sources sharing each sweep, then one sweep per source
(sssp_multi_sweep = 1) with the stored single-source knobs.  Betweenness
centrality ("bc", one source per call) starts from the stored BFS knobs,
searches 2 and 3 for its passes over the levels, then 8 (without bfs_filter)
and 7 for its BFS, which keeps no parents.
The graphs are degree-renumbered on ingest (GR_RENUMBER) unless --no-renumber
is given: the stored knobs serve the layout the benchmark uses.

The tuned values only change the time taken; results are identical for every
setting (the GPU tests check every strategy against the oracle).

CLI:  python -m paper_1701_01170_amd.autotune [--scale 22] [--grid 2048] [--sources 4]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import Graph, default_opts, bc, bfs, bfs_multi, sssp, sssp_multi  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(HERE, "tuning")
ARCH = "gfx950"

KNOBS = ("lb_light_threshold", "lb_chunk", "lb_min_avg_degree", "do_a", "do_b", "device_max_edges",
         "sssp_delta", "adv_block", "twc_wave_min", "twc_block_min", "bfs_filter", "sssp_multi_sweep")
ADV_BLOCK = [128, 256, 512]
TWC_WAVE_MIN = [16, 32, 64, 128, 256]
TWC_BLOCK_MIN = [64, 128, 256, 512, 1024, 4096]
SSSP_DELTA = [0, 8, 16, 32, 64, 128, 256]
SSSP_DELTA_MULTI = [2, 4, 8, 16, 32, 64]
DEVICE_MAX_EDGES = [-1, 1 << 16, 1 << 18, 1 << 20]
MULTI_DO_A = [1 / 4, 1 / 8, 1 / 16, 1 / 32, 1 / 64]
DO_A = [1 / 2, 1 / 4, 1 / 8, 1 / 14, 1 / 32, 1 / 64, 1 / 256]
DO_B = [1 / 576, 1 / 64, 1 / 8]


def graph_class(g: Graph) -> str:
    """'scalefree' when the largest degree dwarfs the average, else 'mesh'."""
    avg = g.n_edges / max(1, g.n_vertices)
    return "scalefree" if g.max_degree > 64 * max(avg, 1.0) else "mesh"


def size_bucket(g: Graph) -> int:
    return int(round(math.log2(max(2, g.n_edges))))


def _path(arch: str = ARCH) -> str:
    return os.path.join(TUNING_DIR, f"{arch}.json")


def load(arch: str = ARCH) -> dict:
    p = _path(arch)
    if not os.path.exists(p):
        return {"arch": arch, "entries": []}
    with open(p) as f:
        return json.load(f)


def lookup(g: Graph, kind: str, arch: str = ARCH) -> dict | None:
    """Best stored knob setting for this graph's class and the nearest size bucket."""
    cls, b = graph_class(g), size_bucket(g)
    cands = [e for e in load(arch)["entries"] if e["class"] == cls and e["kind"] == kind]
    if not cands:
        return None
    return min(cands, key=lambda e: abs(e["log2_edges"] - b))["opts"]


def tuned_opts(g: Graph, kind: str, **overrides):
    """gr_opts with the stored tuned knobs (paper defaults when none stored)."""
    o = default_opts(**overrides)
    t = lookup(g, kind)
    if t:
        for k, v in t.items():
            if k not in overrides:
                setattr(o, k, v)
    return o


def _time(g: Graph, kind: str, sources, knobs: dict, reps: int = 1) -> float:
    import torch
    total = 0.0
    o = default_opts(**knobs)
    if kind in ("bfs_multi", "sssp_multi"):
        srcs = np.asarray(sources, dtype=np.int32)
        run = bfs_multi if kind == "bfs_multi" else sssp_multi
        best = float("inf")
        for _ in range(reps + 1):
            _, _, st = run(g, srcs, opts=o)
            best = min(best, st["device_ms"])
        torch.cuda.synchronize()
        return best
    for s in sources:
        best = float("inf")
        for _ in range(reps + 1):
            if kind == "bfs":
                _, _, st = bfs(g, int(s), opts=o)
            elif kind == "bc":
                _, _, st = bc(g, [int(s)], opts=o)
            else:
                _, _, st = sssp(g, [int(s)], opts=o)
            best = min(best, st["device_ms"])
        total += best
    torch.cuda.synchronize()
    return total / len(sources)


def tune(g: Graph, kind: str, sources, log=print) -> tuple[dict, float, float]:
    """Coordinate descent; returns (best knobs, best ms, paper-default ms)."""
    d = default_opts()
    best = {k: getattr(d, k) for k in KNOBS}
    base_ms = _time(g, kind, sources, best)
    best_ms = base_ms
    log(f"[{kind}] paper defaults: {base_ms:.3f} ms")
    # warm start: the setting already stored for this class (nearest size),
    # since one knob at a time from the defaults can miss a combination
    stored = lookup(g, kind)
    if stored:
        cand = dict(best, **{k: v for k, v in stored.items() if k in KNOBS})
        ms = _time(g, kind, sources, cand)
        log(f"[{kind}] stored setting: {ms:.3f} ms")
        if ms < best_ms * 0.99:
            best, best_ms = cand, ms

    def try_set(key, values, valid=lambda c: True):
        nonlocal best, best_ms
        for v in values:
            cand = dict(best, **{key: v})
            if not valid(cand):
                continue
            ms = _time(g, kind, sources, cand)
            log(f"[{kind}] {key}={v:.6g}: {ms:.3f} ms")
            if ms < best_ms * 0.99:
                best, best_ms = cand, ms

    def tiers_ok(c):
        w, b = c.get("twc_wave_min", 0), c.get("twc_block_min", 0)
        return not (w > 0 and b > 0 and b < w)

    if kind == "sssp_multi":
        # one source per sweep runs the single-source path, whose best knobs
        # are the stored single-source ones; shared sweeps search their own
        try_set("lb_chunk", [512, 1024, 2048])
        try_set("sssp_delta", [0] + SSSP_DELTA_MULTI)
        single = lookup(g, "sssp")
        if single:
            cand = dict(best, **{k: v for k, v in single.items() if k in KNOBS})
            cand["sssp_multi_sweep"] = 1
            ms = _time(g, kind, sources, cand)
            log(f"[{kind}] one source per sweep with the single-source knobs: {ms:.3f} ms")
            if ms < best_ms * 0.99:
                best, best_ms = cand, ms
        return best, best_ms, base_ms
    if kind == "bc":
        # the BFS of each source runs with the stored BFS knobs; the passes
        # over the levels search their LB chunk and workgroup size
        single = lookup(g, "bfs")
        if single:
            cand = dict(best, **{k: v for k, v in single.items() if k in KNOBS})
            ms = _time(g, kind, sources, cand)
            log(f"[{kind}] the BFS knobs: {ms:.3f} ms")
            if ms < best_ms * 0.99:
                best, best_ms = cand, ms
        try_set("lb_chunk", [512, 1024, 2048, 4096, 8192, 16384])
        try_set("adv_block", ADV_BLOCK)
        # its BFS keeps depths only (no parents), so its direction switch
        # and level blocks are searched again
        for a in DO_A:
            for b in DO_B:
                cand = dict(best, do_a=a, do_b=b)
                ms = _time(g, kind, sources, cand)
                log(f"[{kind}] do_a=1/{1 / a:.0f} do_b=1/{1 / b:.0f}: {ms:.3f} ms")
                if ms < best_ms * 0.99:
                    best, best_ms = cand, ms
        try_set("device_max_edges", DEVICE_MAX_EDGES)
        return best, best_ms, base_ms
    try_set("lb_light_threshold", [0, 1024, 4096])
    try_set("lb_chunk", [512, 1024, 2048, 4096, 8192, 16384])
    try_set("adv_block", ADV_BLOCK)
    if kind == "bfs_multi":
        try_set("do_a", MULTI_DO_A)
        return best, best_ms, base_ms
    try_set("lb_min_avg_degree", [0.0, 5.0, 1e9])
    if g.n_edges < best["lb_min_avg_degree"] * g.n_vertices:  # TWC expands the push levels
        try_set("twc_wave_min", TWC_WAVE_MIN, tiers_ok)
        try_set("twc_block_min", TWC_BLOCK_MIN, tiers_ok)
    if kind == "sssp":
        try_set("sssp_delta", SSSP_DELTA)
    try_set("device_max_edges", DEVICE_MAX_EDGES)
    if kind == "bfs":
        for a in DO_A:
            for b in DO_B:
                cand = dict(best, do_a=a, do_b=b)
                ms = _time(g, kind, sources, cand)
                log(f"[{kind}] do_a=1/{1 / a:.0f} do_b=1/{1 / b:.0f}: {ms:.3f} ms")
                if ms < best_ms * 0.99:
                    best, best_ms = cand, ms
        try_set("bfs_filter", [0, 1, 2])
    return best, best_ms, base_ms


def store(g: Graph, kind: str, knobs: dict, best_ms: float, base_ms: float, graph_name: str,
          sources, arch: str = ARCH) -> None:
    os.makedirs(TUNING_DIR, exist_ok=True)
    db = load(arch)
    cls, b = graph_class(g), size_bucket(g)
    db["entries"] = [e for e in db["entries"]
                     if not (e["class"] == cls and e["kind"] == kind and e["log2_edges"] == b)]
    db["entries"].append({"class": cls, "kind": kind, "log2_edges": b, "graph": graph_name,
                          "sources": [int(s) for s in sources], "opts": knobs,
                          "device_ms": round(best_ms, 4), "paper_default_ms": round(base_ms, 4),
                          "date": time.strftime("%Y-%m-%d")})
    db["entries"].sort(key=lambda e: (e["class"], e["kind"], e["log2_edges"]))
    with open(_path(arch), "w") as f:
        json.dump(db, f, indent=1)


def main():
    from . import Context
    from . import graphgen as gg
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, nargs="*", default=[22])
    ap.add_argument("--grid", type=int, nargs="*", default=[])
    ap.add_argument("--sources", type=int, default=4)
    ap.add_argument("--kinds", default="bfs,sssp")
    ap.add_argument("--no-renumber", action="store_true",
                    help="tune on graphs in generation order instead of degree-renumbered ones")
    args = ap.parse_args()
    ctx = Context(0)
    graphs = [(f"rmat_s{s}_e16", gg.add_weights(gg.rmat(s, 16, seed=1), seed=101)) for s in args.scale]
    graphs += [(f"grid_{n}x{n}", gg.add_weights(gg.grid(n, n), seed=101)) for n in args.grid]
    for name, hg in graphs:
        g = Graph.from_host(ctx, hg, symmetric=True, renumber=not args.no_renumber)
        srcs = gg.sources(hg, args.sources, seed=2000)  # held-out from the bench's sources
        for kind in args.kinds.split(","):
            ks = (gg.sources(hg, 64, seed=2100) if kind == "bfs_multi" else
                  gg.sources(hg, 16, seed=2200) if kind == "sssp_multi" else srcs)
            knobs, ms, base = tune(g, kind, ks, log=lambda m: print(f"{name} {m}", flush=True))
            store(g, kind, knobs, ms, base, name, ks)
            print(f"{name} [{kind}] best {ms:.3f} ms (paper defaults {base:.3f} ms): {knobs}", flush=True)
        g.free()


if __name__ == "__main__":
    main()
