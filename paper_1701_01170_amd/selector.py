"""Training and evaluation of the learned strategy selector.

Traces: the traversals themselves record, for every iteration, the eight
selector features, the action taken and its event-timed step time
(gr_level_trace).  Because the filter is exact, the frontier of every level is
the same whatever actions were taken, so runs with each fixed action and with
seeded random actions observe every action's time at the same levels (with
both "previous step pushed" and "previous step pulled" states).  Each record
becomes one training sample whose target is log2(step time in us) for the
action taken, with the other three outputs masked out.  The mask carries a
sample weight so that every (graph, traversal) pair weighs the same in the
loss (a 2048 x 2048 grid yields thousands of levels, an R-MAT graph a dozen).

Training runs on the GPU with the library's own kernels (gr_mlp_loss_grad,
gr_mlp_adam); evaluation compares event-timed traversal time with the
heuristic and with the network on held-out sources.

A second network serves the batched BFS (gr_bfs_multi, 64 sources per
pass): its traces come from batched runs with each fixed action and with
seeded random actions, its features are the same eight with the unvisited
counts averaged over the pass's sources.  Both networks are loaded together
(gr_ctx_set_policy with 2 x 1476 parameters, see load_policy).

Graphs are ingested degree-renumbered (GR_RENUMBER), the layout the benchmark
and the tuner use, unless --no-renumber is given.

CLI:  python -m paper_1701_01170_amd.selector [--quick] [--epochs N]
      python -m paper_1701_01170_amd.selector --multi [--quick] [--epochs N]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import (MLP_N_PARAMS, POLICY_FIXED, POLICY_HEURISTIC, POLICY_LEARNED, POLICY_RANDOM,
               Context, Graph, LevelTrace, bfs, bfs_multi, default_opts, mlp_adam, mlp_loss_grad,
               sssp)
from . import graphgen as gg

RENUMBER = True  # ingest the traces' graphs degree-renumbered

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "tuning", "selector_gfx950.npy")
REPORT = os.path.join(HERE, "tuning", "selector_gfx950.json")
WEIGHTS_MULTI = os.path.join(HERE, "tuning", "selector_multi_gfx950.npy")
REPORT_MULTI = os.path.join(HERE, "tuning", "selector_multi_gfx950.json")


def load_policy(ctx: Context) -> bool:
    """Load the trained networks into ctx: the single-source one, followed by
    the batched-BFS one when it exists.  False when no weights are stored."""
    if not os.path.exists(WEIGHTS):
        return False
    p = np.load(WEIGHTS).astype(np.float32)
    if os.path.exists(WEIGHTS_MULTI):
        p = np.concatenate([p, np.load(WEIGHTS_MULTI).astype(np.float32)])
    ctx.set_policy(p)
    return True


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initialisation in the documented flat layout."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((32, 8)) * np.sqrt(2 / 8), np.zeros(32),
             rng.standard_normal((32, 32)) * np.sqrt(2 / 32), np.zeros(32),
             rng.standard_normal((4, 32)) * np.sqrt(1 / 32), np.full(4, 6.0)]
    flat = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert flat.shape[0] == MLP_N_PARAMS
    return flat


def _records(buf, count):
    out = []
    for t in buf[:count]:
        if t.step_us > 0:
            out.append((list(t.features), t.action, float(t.step_us)))
    return out


def collect(ctx: Context, graphs, n_sources: int = 3, random_runs: int = 4, sssp_too: bool = True,
            log=print):
    """Trace samples X[n][8], T[n][4], M[n][4] from fixed- and random-action runs."""
    cap = 1 << 15
    buf = (LevelTrace * cap)()
    X, T, M, grp = [], [], [], []

    def add(recs, group):
        for f, a, us in recs:
            X.append(f)
            t = np.zeros(4, np.float32)
            m = np.zeros(4, np.float32)
            t[a] = np.log2(us)
            m[a] = 1.0
            T.append(t)
            M.append(m)
            grp.append(group)

    from . import autotune
    for name, hg in graphs:
        t0 = time.time()
        g = Graph.from_host(ctx, hg, symmetric=True, renumber=RENUMBER)
        # R-MAT graphs (the workload the selector serves first) get more sources
        srcs = gg.sources(hg, 2 * n_sources if name.startswith("rmat") else n_sources, seed=3000)
        # the tuned chunk sizes and thresholds of this graph's class, and one
        # host round trip per level (no device-predicated blocks), so that
        # every record times exactly one step of the action it names
        pols = [dict(policy=POLICY_FIXED, fixed_action=a, device_max_edges=-1) for a in range(4)]
        pols += [dict(policy=POLICY_RANDOM, policy_seed=100 + r, device_max_edges=-1)
                 for r in range(random_runs)]
        for s in srcs:
            for kw in pols:
                o = autotune.tuned_opts(g, "bfs", trace=buf, trace_capacity=cap, **kw)
                bfs(g, int(s), opts=o)
                add(_records(buf, min(o.trace_count, cap)), name + "/bfs")
                if sssp_too and hg.weights is not None and kw["policy"] != POLICY_RANDOM and \
                        kw.get("fixed_action", 0) < 2:
                    o = autotune.tuned_opts(g, "sssp", trace=buf, trace_capacity=cap, **kw)
                    sssp(g, [int(s)], opts=o)
                    add(_records(buf, min(o.trace_count, cap)), name + "/sssp")
        g.free()
        log(f"traced {name}: {len(X)} samples so far ({time.time() - t0:.1f}s)")
    M = np.asarray(M, np.float32)
    _, inv, counts = np.unique(np.asarray(grp), return_inverse=True, return_counts=True)
    w = len(grp) / (len(counts) * counts[inv])
    M *= w[:, None].astype(np.float32)
    return (np.asarray(X, np.float32), np.asarray(T, np.float32), M)


def collect_multi(ctx: Context, graphs, ks=(16, 64), random_runs: int = 4, log=print):
    """Samples from batched BFS runs (k sources for each k in ks) with each
    fixed action and with seeded random actions, one host round trip per
    level, so every record times one level of the action it names."""
    from . import autotune
    cap = 1 << 15
    buf = (LevelTrace * cap)()
    X, T, M, grp = [], [], [], []
    for name, hg in graphs:
        t0 = time.time()
        g = Graph.from_host(ctx, hg, symmetric=True, renumber=RENUMBER)
        pols = [dict(policy=POLICY_FIXED, fixed_action=a) for a in (0, 1, 2)]
        pols += [dict(policy=POLICY_RANDOM, policy_seed=100 + r) for r in range(random_runs)]
        for k in ks:
            srcs = gg.sources(hg, k, seed=3000).astype(np.int32)
            for kw in pols:
                o = autotune.tuned_opts(g, "bfs_multi", trace=buf, trace_capacity=cap, **kw)
                bfs_multi(g, srcs, opts=o)
                for f, a, us in _records(buf, min(o.trace_count, cap)):
                    X.append(f)
                    t = np.zeros(4, np.float32)
                    m = np.zeros(4, np.float32)
                    t[a] = np.log2(us)
                    m[a] = 1.0
                    T.append(t)
                    M.append(m)
                    grp.append(f"{name}/k{k}")
        g.free()
        log(f"traced batched {name}: {len(X)} samples so far ({time.time() - t0:.1f}s)")
    M = np.asarray(M, np.float32)
    _, inv, counts = np.unique(np.asarray(grp), return_inverse=True, return_counts=True)
    w = len(grp) / (len(counts) * counts[inv])
    M *= w[:, None].astype(np.float32)
    return (np.asarray(X, np.float32), np.asarray(T, np.float32), M)


def evaluate_multi(ctx: Context, graphs, params_multi, ks=(16, 64), reps: int = 3,
                   margins=(0.0,), log=print) -> list[dict]:
    """Batched BFS (k sources) under the heuristic and under the batched
    network, tuned knobs, best of `reps` device times each."""
    from . import autotune
    single = np.load(WEIGHTS).astype(np.float32) if os.path.exists(WEIGHTS) else \
        np.zeros(MLP_N_PARAMS, np.float32)
    ctx.set_policy(np.concatenate([single, params_multi.astype(np.float32)]))
    rows = []
    try:
        for name, hg in graphs:
            g = Graph.from_host(ctx, hg, symmetric=True, renumber=RENUMBER)
            for k in ks:
                srcs = gg.sources(hg, k, seed=9100).astype(np.int32)
                cfgs = {"heuristic": autotune.tuned_opts(g, "bfs_multi")}
                for mg in margins:
                    cfgs[f"learned_margin{mg:g}"] = autotune.tuned_opts(
                        g, "bfs_multi", policy=POLICY_LEARNED, learned_margin=mg)
                res = {}
                for label, o in cfgs.items():
                    best, st = float("inf"), None
                    for _ in range(reps):
                        st = bfs_multi(g, srcs, opts=o)[2]
                        best = min(best, st["device_ms"])
                    res[label] = dict(ms=round(best, 4),
                                      gteps=round(st["teps_edges"] / (best * 1e-3) / 1e9, 3),
                                      actions=st["action_count"])
                row = dict(graph=name, kind="bfs_multi", k=k, **res)
                rows.append(row)
                log(json.dumps(row))
            g.free()
    finally:
        ctx.set_policy(None)
    return rows


def training_graphs_multi(quick: bool):
    """R-MAT scales 16..22 with a in [0.45, 0.65] and scale 24 with the
    paper's a, Erdos-Renyi average degree 4..64, grids 256^2 and 512^2
    (batched runs over the larger grids take thousands of levels per source
    pass)."""
    gs = []
    for s in ([16, 18] if quick else [16, 18, 20, 22]):
        for a in (0.45, 0.55, 0.65):
            gs.append((f"rmat_s{s}_a{a}", gg.rmat_family(s, 16, a, seed=11 + s)))
    if not quick:
        gs.append(("rmat_s24_a0.57", gg.rmat(24, 16, seed=35)))
    for d in ((4, 64) if quick else (4, 16, 64)):
        gs.append((f"er_n262144_d{d}", gg.erdos_renyi(1 << 18, d, seed=5)))
    for n in (256, 512):
        gs.append((f"grid_{n}", gg.grid(n, n)))
    return gs


def eval_graphs_multi():
    return [("rmat_s22_e16", gg.rmat(22, 16, seed=1)),
            ("rmat_s20_e16", gg.rmat(20, 16, seed=1)),
            ("rmat_s18_e16_seed3", gg.rmat(18, 16, seed=3)),
            ("er_n262144_d8", gg.erdos_renyi(1 << 18, 8, seed=77)),
            ("grid_384", gg.grid(384, 384))]


def train(ctx: Context, X, T, M, epochs: int = 400, lr: float = 3e-3, seed: int = 0, log=print):
    """Full-batch Adam on the GPU kernels; returns float32 parameters."""
    import torch
    dX = torch.from_numpy(X).cuda()
    dT = torch.from_numpy(T).cuda()
    dM = torch.from_numpy(M).cuda()
    p = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    grad = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for step in range(1, epochs + 1):
        mlp_loss_grad(ctx, p, dX, dT, dM, grad=grad, loss=loss)
        mlp_adam(ctx, p, grad, m, v, step, lr=lr)
        if step == 1 or step % 100 == 0 or step == epochs:
            log(f"step {step}: loss {loss.item():.4f}")
    return p.cpu().numpy()


def evaluate(ctx: Context, graphs, params, n_sources: int = 5, margins=(0.0,),
             log=print) -> list[dict]:
    """Median device time of BFS and SSSP under the heuristic (paper defaults
    and autotuned knobs) and under the network, on held-out sources."""
    from . import autotune
    ctx.set_policy(params)
    rows = []
    try:
        for name, hg in graphs:
            g = Graph.from_host(ctx, hg, symmetric=True, renumber=RENUMBER)
            srcs = gg.sources(hg, n_sources, seed=9000)
            for kind in ("bfs", "sssp"):
                if kind == "sssp" and hg.weights is None:
                    continue
                res = {}
                # the network chooses the action; chunk sizes and thresholds are
                # the tuned ones in both tuned configurations
                cfgs = {"heuristic_paper_knobs": default_opts(),
                        "heuristic_tuned_knobs": autotune.tuned_opts(g, kind)}
                for mg in margins:
                    cfgs[f"learned_tuned_knobs_margin{mg:g}"] = autotune.tuned_opts(
                        g, kind, policy=POLICY_LEARNED, learned_margin=mg)
                for label, o in cfgs.items():
                    times, teps = [], []
                    for s in srcs:
                        best = float("inf")
                        for _ in range(3):
                            if kind == "bfs":
                                st = bfs(g, int(s), opts=o)[2]
                            else:
                                st = sssp(g, [int(s)], opts=o)[2]
                            best = min(best, st["device_ms"])
                        times.append(best)
                        teps.append(st["teps_edges"])
                    # GTEPS of the summed work over the summed best times
                    res[label] = dict(ms=round(float(np.median(times)), 4),
                                      gteps=round(sum(teps) / (sum(times) * 1e-3) / 1e9, 3))
                row = dict(graph=name, kind=kind, **res)
                rows.append(row)
                log(json.dumps(row))
            g.free()
    finally:
        ctx.set_policy(None)
    return rows


def training_graphs(quick: bool):
    """Synthetic training set: R-MAT scales 16..22 with a in [0.45, 0.65]
    (b:c:d kept) and scale 24 with the paper's a, Erdos-Renyi average degree
    4..64, grids 256^2..2048^2."""
    gs = []
    scales = [16, 18] if quick else [16, 18, 20, 22]
    for s in scales:
        for a in (0.45, 0.55, 0.65):
            gs.append((f"rmat_s{s}_a{a}", gg.add_weights(gg.rmat_family(s, 16, a, seed=11 + s), seed=7)))
    if not quick:
        gs.append(("rmat_s24_a0.57", gg.add_weights(gg.rmat(24, 16, seed=35), seed=7)))
    for d in ((4, 64) if quick else (4, 16, 64)):
        gs.append((f"er_n262144_d{d}", gg.add_weights(gg.erdos_renyi(1 << 18, d, seed=5), seed=7)))
    for n in ((256, 512) if quick else (256, 512, 1024, 2048)):
        gs.append((f"grid_{n}", gg.add_weights(gg.grid(n, n), seed=7)))
    return gs


def eval_graphs():
    """Held-out: the scale-14 R-MAT of the small BFS workload (seed 1, the
    paper's initiator) plus graphs of the other classes with unseen seeds."""
    return [("rmat_s14_e16", gg.add_weights(gg.rmat(14, 16, seed=1), seed=101)),
            ("rmat_s20_e16", gg.add_weights(gg.rmat(20, 16, seed=3), seed=101)),
            ("er_n262144_d8", gg.add_weights(gg.erdos_renyi(1 << 18, 8, seed=77), seed=101)),
            ("grid_768", gg.add_weights(gg.grid(768, 768), seed=101))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--sources", type=int, default=3)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the stored weights")
    ap.add_argument("--margins", default="0,0.1,0.25,0.5")
    ap.add_argument("--multi", action="store_true", help="train the batched-BFS network")
    ap.add_argument("--no-renumber", action="store_true",
                    help="ingest the graphs in generation order instead of degree-renumbered")
    args = ap.parse_args()
    global RENUMBER
    RENUMBER = not args.no_renumber
    margins = [float(x) for x in args.margins.split(",")]
    ctx = Context(0)
    if args.multi:
        log = lambda m: print(m, flush=True)  # noqa: E731
        t0 = time.time()
        X, T, M = collect_multi(ctx, training_graphs_multi(args.quick), log=log)
        print(f"collected {X.shape[0]} batched samples in {time.time() - t0:.1f}s", flush=True)
        params = train(ctx, X, T, M, epochs=args.epochs, log=log)
        os.makedirs(os.path.dirname(WEIGHTS_MULTI), exist_ok=True)
        np.save(WEIGHTS_MULTI, params.astype(np.float32))
        rows = evaluate_multi(ctx, eval_graphs_multi(), params, margins=margins, log=log)
        with open(REPORT_MULTI, "w") as f:
            json.dump(dict(samples=int(X.shape[0]), epochs=args.epochs, eval=rows), f, indent=1)
        return
    if args.eval_only:
        rows = evaluate(ctx, eval_graphs(), np.load(WEIGHTS), margins=margins,
                        log=lambda s: print(s, flush=True))
        with open(REPORT) as f:
            rep = json.load(f)
        rep["eval"] = rows
        with open(REPORT, "w") as f:
            json.dump(rep, f, indent=1)
        return
    t0 = time.time()
    X, T, M = collect(ctx, training_graphs(args.quick), n_sources=args.sources,
                      log=lambda s: print(s, flush=True))
    print(f"collected {X.shape[0]} samples in {time.time() - t0:.1f}s", flush=True)
    params = train(ctx, X, T, M, epochs=args.epochs, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(WEIGHTS), exist_ok=True)
    np.save(WEIGHTS, params.astype(np.float32))
    rows = evaluate(ctx, eval_graphs(), params, margins=margins, log=lambda s: print(s, flush=True))
    with open(REPORT, "w") as f:
        json.dump(dict(samples=int(X.shape[0]), epochs=args.epochs, eval=rows), f, indent=1)


if __name__ == "__main__":
    main()
