#!/usr/bin/env python3
"""Benchmark of PR-Nibble + sweep cut on one MI355X.

Workload (default, "plain22"): undirected R-MAT graph (a,b,c,d) =
(0.57,0.19,0.19,0.05), 2^22 vertices, 16 * 2^22 edge samples (avg degree ~31
after symmetrising and removing self-loops and duplicates), int32 ids with
int64 offsets; 16 seeds drawn uniformly from vertices of degree >= 1, run one
after another (alpha = 0.01, eps = 1e-7, optimized push rule, FP64 p and r).
A step is those 16 queries, each a full PR-Nibble push followed by the sweep
cut, with the graph already resident in HBM.

Prints one JSON line: pushed edges/s (value), queries/s, per-query latency
p50/p99, the HBM-roofline fraction of the edge-scatter kernel (HIP events on
the library's stream, summed over the timed steps), and the oracle timed on a
bounded sample on the host as a CPU baseline.
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

WORKLOADS = {
    # 16 seeds one after another on the 2^22 graph (plain path)
    "plain22": dict(scale=22, ef=16, nseeds=16, alpha=0.01, eps=1e-7, batched=False),
    # the 2^16 graph from vertex 0 of the largest component
    "plain16": dict(scale=16, ef=8, nseeds=1, alpha=0.01, eps=1e-7, batched=False),
    # 256 seeds in one batch on the 2^22 graph, eps log-uniform in [1e-7, 1e-5],
    # alpha in {0.01, 0.05}
    "batched22": dict(scale=22, ef=16, nseeds=256, eps_lo=1e-7, eps_hi=1e-5, batched=True,
                      slots=256),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain22", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(seeds would shard across GPUs, one graph replica each); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1604_07515_amd as plc

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    g = synth.rmat(wl["scale"], wl["ef"], seed=1)
    if wl["batched"]:
        qs = synth.batched_queries(g, wl["nseeds"], seed=2, eps_lo=wl["eps_lo"],
                                   eps_hi=wl["eps_hi"])
        seeds, alphas, epss = qs.seeds, qs.alpha, qs.eps
    else:
        if args.workload == "plain16":
            seeds = np.array([synth.largest_component_min_vertex(g)], np.int32)
        else:
            seeds = synth.uniform_seeds(g, wl["nseeds"], seed=2)
        alphas = np.full(len(seeds), wl["alpha"])
        epss = np.full(len(seeds), wl["eps"])
    log("graph n=%d arcs=%d maxdeg=%d (%.1fs)" % (g.n, g.arcs, g.deg.max(), time.time() - t0))

    arena = plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20)
    if wl["batched"]:
        arena += plc.batch_arena_bytes(g.n, g.arcs, wl["slots"])
    ctx = plc.Context(arena_bytes=arena, device=0)
    hg = ctx.load_graph(g.off, g.nbr)
    if wl["batched"]:
        got = ctx.batch_reserve(hg, wl["slots"])
        log("batch slots granted: %d" % got)

    def step(lat, acc):
        if wl["batched"]:
            q0 = time.perf_counter()
            ids, infos = ctx.run_batched(hg, seeds, alphas, epss)
            lat.append(time.perf_counter() - q0)
        else:
            ids, infos = [], []
            for s, al, ep in zip(seeds, alphas, epss):
                q0 = time.perf_counter()
                i1, f1 = ctx.run(hg, [int(s)], float(al), float(ep))
                lat.append(time.perf_counter() - q0)
                ids += i1
                infos += f1
        for qid, info in zip(ids, infos):
            acc["edges"] += info["edges"]
            acc["pushes"] += info["pushes"]
            acc["rounds"] += info["rounds"]
            acc["support"] += info["support"]
            ctx.release(qid)

    for i in range(args.warmup):
        step([], {"edges": 0, "pushes": 0, "rounds": 0, "support": 0})
        log("warmup step %d done" % i)
    torch.cuda.synchronize()
    ctx.timing(True)
    lat = []
    acc = {"edges": 0, "pushes": 0, "rounds": 0, "support": 0}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(lat, acc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    tm = ctx.timing_get()
    ctx.timing(False)
    log("timed %d steps in %.3fs" % (args.steps, elapsed))

    nq = args.steps * len(seeds)
    edges_per_s = acc["edges"] / elapsed
    sc = tm["scatter"]
    scatter_bytes = SCATTER_B_PER_EDGE * sc["units"] + SCATTER_B_PER_ENTRY * sc["entries"]
    scatter_gbs = scatter_bytes / (sc["ms"] * 1e-3) / 1e9 if sc["ms"] > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": edges_per_s,
        "unit": "pushed edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "rmat%d_ef%d_%s_%dseeds" % (wl["scale"], wl["ef"],
                                                     "batched" if wl["batched"] else "plain",
                                                     len(seeds)),
            "n": g.n, "arcs": g.arcs, "rule": "optimized", "queries_per_step": len(seeds),
            "alpha": sorted(set(float(x) for x in alphas)),
            "eps": [float(epss.min()), float(epss.max())],
            "path": ("batched (%d slots, one round of every query per launch)" % wl["slots"]
                     if wl["batched"] else "plain (one query at a time)"),
        },
        "queries_per_s": nq / elapsed,
        "latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3,
                       "what": "per batch call" if wl["batched"] else "per query"},
        "per_query": {"edges": acc["edges"] / nq, "pushes": acc["pushes"] / nq,
                      "rounds": acc["rounds"] / nq, "support": acc["support"] / nq},
        "kernels": tm,
        "roofline": {
            "kernel": "k_scatter",
            "bound": "hbm",
            "achieved": scatter_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": scatter_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_model": "20 B per pushed edge + 24 B per pushed vertex",
            "avg_launch_us": sc["ms"] * 1e3 / max(sc["launches"], 1),
        },
    }

    if args.cpu_budget > 0:
        import oracle
        budget = args.cpu_budget
        c0 = time.perf_counter()
        done, e_sum = 0, 0
        for s, al, ep in zip(seeds, alphas, epss):
            r = oracle.prnibble(g.off, g.nbr, int(s), float(al), float(ep))
            oracle.sweep(g.off, g.nbr, r.p)
            done += 1
            e_sum += r.edges
            if time.perf_counter() - c0 > budget:
                break
        ct = time.perf_counter() - c0
        out["cpu_baseline"] = {
            "value": e_sum / ct, "unit": "pushed edges/s", "cores": 1, "kind": "oracle",
            "queries_per_s": done / ct,
            "sample": "first %d of the %d seeds of one step, single-threaded oracle "
                      "(push + sweep), %.1f s" % (done, len(seeds), ct),
        }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
