#!/usr/bin/env python3
"""Benchmark of PR-Nibble + sweep cut on one MI355X.

Default run (about two minutes): three workloads on synthetic undirected
R-MAT graphs, (a,b,c,d) = (0.57,0.19,0.19,0.05), edge factor 16 (average
degree ~31 after symmetrising and removing self-loops and duplicates),
int32 ids, int64 offsets, FP64 p and r, optimized push rule:

* plain22 (the line's `value`): 2^22 vertices, 16 seeds drawn uniformly
  from vertices of degree >= 1, run one after another, alpha = 0.01,
  eps = 1e-7.  A step is those 16 queries, each a full PR-Nibble push
  followed by the sweep cut, graph resident in HBM.
* batched22: the same graph, 256 seeds in one batch (256 slots), eps
  log-uniform in [1e-7, 1e-5], alpha in {0.01, 0.05}; a step is the batch.
* serve24: 2^24 vertices, seeds drawn proportionally to degree, eps
  log-uniform in [1e-7, 1e-4], alpha = 0.01, continuous batching over 64
  slots: the saturation rate (all queries queued at once) and Poisson
  arrivals at 50% and 90% of it, with p50/p99 latency.

Prints one JSON line.  The roofline object describes the edge-scatter
kernel, timed with HIP events on the library's stream over the timed steps.
The CPU baseline is the oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PR-Nibble+sweep edges/s & queries/s (batched vs plain); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the edge scatter: per pushed edge the neighbour id
# (4 B) and a read and a write of r[w] (8 + 8 B); per pushed vertex the staged
# entry (edge start 8 B, row offset 8 B, coefficient 8 B).
SCATTER_B_PER_EDGE = 20
SCATTER_B_PER_ENTRY = 24


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def roofline(tm):
    sc = tm["scatter"]
    by = SCATTER_B_PER_EDGE * sc["units"] + SCATTER_B_PER_ENTRY * sc["entries"]
    gbs = by / (sc["ms"] * 1e-3) / 1e9 if sc["ms"] > 0 else 0.0
    return {
        "kernel": "scatter (edgeMap UpdateNgh)", "bound": "hbm", "achieved": gbs,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
        "bytes_model": "20 B per pushed edge + 24 B per pushed vertex",
        "launches": sc["launches"], "avg_launch_us": sc["ms"] * 1e3 / max(sc["launches"], 1),
        "edges_per_s": sc["units"] / (sc["ms"] * 1e-3) if sc["ms"] > 0 else 0.0,
    }


def timed_steps(ctx, step, steps, warmup):
    import torch
    acc = {"edges": 0, "pushes": 0, "rounds": 0, "support": 0, "queries": 0}
    for i in range(warmup):
        step([], dict(acc))
        log("  warmup step %d done" % i)
    torch.cuda.synchronize()
    ctx.timing(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(lat, acc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = ctx.timing_get()
    ctx.timing(False)
    return elapsed, lat, acc, tm


def account(acc, infos, ids, ctx):
    for qid, info in zip(ids, infos):
        acc["edges"] += info["edges"]
        acc["pushes"] += info["pushes"]
        acc["rounds"] += info["rounds"]
        acc["support"] += info["support"]
        acc["queries"] += 1
        ctx.release(qid)


def bench_plain(plc, synth, g, steps, warmup):
    import numpy as np
    seeds = synth.uniform_seeds(g, 16, seed=2)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    tune = ctx.autotune(hg, seeds, 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
    log("  plain launch shapes: self %d, scatter %d, sweep %d workgroups (%d tried)" % (
        tune["plain_self"], tune["plain_scatter"], tune["plain_sweep"], tune["candidates"]))

    def step(lat, acc):
        for s in seeds:
            q0 = time.perf_counter()
            ids, infos = ctx.run(hg, [int(s)], 0.01, 1e-7)
            lat.append(time.perf_counter() - q0)
            account(acc, infos, ids, ctx)

    elapsed, lat, acc, tm = timed_steps(ctx, step, steps, warmup)
    ctx.close()
    nq = acc["queries"]
    return {
        "seeds": seeds, "elapsed": elapsed, "edges_per_s": acc["edges"] / elapsed,
        "queries_per_s": nq / elapsed, "ms_per_step": elapsed * 1e3 / steps,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3, "what": "per query"},
        "per_query": {k: acc[k] / nq for k in ("edges", "pushes", "rounds", "support")},
        "kernels": tm, "roofline": roofline(tm),
        "launch_shapes": {k: tune[k] for k in ("plain_self", "plain_scatter", "plain_sweep")},
    }


def bench_batched(plc, synth, g, steps, warmup, slots=256):
    qs = synth.batched_queries(g, 256, seed=2, eps_lo=1e-7, eps_hi=1e-5)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, slots) + (512 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    got = ctx.batch_reserve(hg, slots)
    tune = ctx.autotune(hg, qs.seeds, qs.alpha, qs.eps, plc.PLC_TUNE_BATCH)
    log("  batched launch shapes: self %d, scatter %d workgroups (%d tried)" % (
        tune["batch_self"], tune["batch_scatter"], tune["candidates"]))

    def step(lat, acc):
        q0 = time.perf_counter()
        ids, infos = ctx.run_batched(hg, qs.seeds, qs.alpha, qs.eps)
        lat.append(time.perf_counter() - q0)
        account(acc, infos, ids, ctx)

    elapsed, lat, acc, tm = timed_steps(ctx, step, steps, warmup)
    ctx.close()
    nq = acc["queries"]
    return {
        "queries": qs, "workload": "rmat%d_ef16_batched_256seeds" % (g.n.bit_length() - 1),
        "slots": got, "edges_per_s": acc["edges"] / elapsed, "queries_per_s": nq / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "what": "per batch of 256"},
        "per_query": {k: acc[k] / nq for k in ("edges", "pushes", "rounds", "support")},
        "eps": [float(qs.eps.min()), float(qs.eps.max())], "alpha": [0.01, 0.05],
        "kernels": tm, "roofline": roofline(tm),
        "launch_shapes": {k: tune[k] for k in ("batch_self", "batch_scatter", "batch_sweep")},
    }


def bench_serving(plc, synth, scale, nq, slots=64):
    import numpy as np
    from paper_1604_07515_amd import serve
    t0 = time.time()
    g = synth.rmat(scale, 16, seed=1)
    log("serving graph 2^%d: n=%d arcs=%d (%.1fs)" % (scale, g.n, g.arcs, time.time() - t0))
    rng = np.random.default_rng(2)
    seeds = synth.degree_weighted_seeds(g, nq, rng)
    eps = 10.0 ** rng.uniform(-7, -4, nq)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, slots) + (1 << 30))
    hg = ctx.load_graph(g.off, g.nbr)
    got = ctx.batch_reserve(hg, slots)
    ctx.autotune(hg, seeds[:128], 0.01, eps[:128], plc.PLC_TUNE_BATCH)
    serve.saturation(ctx, hg, seeds[:256], 0.01, eps[:256])  # warm-up
    sat = serve.saturation(ctx, hg, seeds, 0.01, eps)
    out = {"workload": "rmat%d_ef16_serving_poisson" % scale, "n": g.n, "arcs": g.arcs,
           "slots": got, "queries_per_run": nq, "alpha": 0.01, "eps": [1e-7, 1e-4],
           "seeds": "proportional to degree",
           "saturation": {"queries_per_s": sat.queries_per_s,
                          "edges_per_s": sat.edges / sat.wall_s,
                          "p50_ms": sat.percentile_ms(50), "p99_ms": sat.percentile_ms(99)},
           "poisson": []}
    for frac in (0.5, 0.9):
        qps = frac * sat.queries_per_s
        arr = serve.poisson_arrivals(nq, qps, np.random.default_rng(3))
        rep = serve.serve(ctx, hg, seeds, 0.01, eps, arr)
        out["poisson"].append({"offered_qps": qps, "served_qps": rep.queries_per_s,
                               "p50_ms": rep.percentile_ms(50), "p99_ms": rep.percentile_ms(99),
                               "max_in_flight": rep.max_in_flight})
        log("  poisson %.0f qps: p50 %.2f ms p99 %.2f ms" % (qps, rep.percentile_ms(50),
                                                            rep.percentile_ms(99)))
    ctx.close()
    return out


def cpu_baseline(oracle, g, work, budget):
    """The oracle, single-threaded, on the first queries of the workload list."""
    c0 = time.perf_counter()
    done = e_sum = 0
    for s, al, ep in work:
        r = oracle.prnibble(g.off, g.nbr, int(s), float(al), float(ep))
        oracle.sweep(g.off, g.nbr, r.p)
        done += 1
        e_sum += r.edges
        if time.perf_counter() - c0 > budget:
            break
    ct = time.perf_counter() - c0
    return {"value": e_sum / ct, "unit": "pushed edges/s", "cores": 1, "kind": "oracle",
            "queries_per_s": done / ct,
            "sample": "%d queries (the 16 plain seeds, then the batched seeds in order), "
                      "single-threaded oracle push + sweep, %.1f s" % (done, ct)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=["plain", "batched", "serving"], default=None,
                    help="run one workload only (the others are reported as skipped)")
    ap.add_argument("--serve-scale", type=int, default=24)
    ap.add_argument("--serve-queries", type=int, default=2048)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(seeds would shard across GPUs, one graph replica each); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import synth
    import paper_1604_07515_amd as plc

    t0 = time.time()
    g = synth.rmat(22, 16, seed=1)
    log("graph 2^22: n=%d arcs=%d maxdeg=%d (%.1fs)" % (g.n, g.arcs, g.deg.max(), time.time() - t0))
    want = lambda w: args.only is None or args.only == w
    plain = bench_plain(plc, synth, g, args.steps, args.warmup) if want("plain") else None
    if plain:
        log("plain: %.3g edges/s, %.1f queries/s" % (plain["edges_per_s"], plain["queries_per_s"]))
    bat = bench_batched(plc, synth, g, max(2, args.steps // 2), 1) if want("batched") else None
    if bat:
        log("batched: %.3g edges/s, %.1f queries/s" % (bat["edges_per_s"], bat["queries_per_s"]))
    srv = bench_serving(plc, synth, args.serve_scale, args.serve_queries) if want("serving") else None

    main_res = plain or bat
    out = {
        "metric": METRIC,
        "value": main_res["edges_per_s"] if main_res else None,
        "unit": "pushed edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"] if main_res else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": ({"workload": "rmat22_ef16_plain_16seeds", "n": g.n, "arcs": g.arcs,
                    "alpha": 0.01, "eps": 1e-7, "rule": "optimized", "queries_per_step": 16,
                    "path": "plain (one query at a time)"} if plain else
                   {"workload": bat["workload"], "n": g.n, "arcs": g.arcs}),
    }
    if main_res:
        out["queries_per_s"] = main_res["queries_per_s"]
        out["latency_ms"] = main_res["latency_ms"]
        out["per_query"] = main_res["per_query"]
        out["roofline"] = main_res["roofline"]
        out["kernels"] = main_res["kernels"]
    if bat:
        out["batched"] = {k: v for k, v in bat.items() if k != "queries"}
        if plain:
            out["batched"]["queries_per_s_vs_plain"] = bat["queries_per_s"] / plain["queries_per_s"]
    if srv:
        out["serving"] = srv
    if args.cpu_budget > 0:
        import oracle
        work = []
        if plain:
            work += [(s, 0.01, 1e-7) for s in plain["seeds"]]
        if bat:
            q = bat["queries"]
            work += list(zip(q.seeds, q.alpha, q.eps))
        if work:
            out["cpu_baseline"] = cpu_baseline(oracle, g, work, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
