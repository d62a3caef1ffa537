#!/usr/bin/env python3
"""Benchmark of PR-Nibble + sweep cut on one MI355X.

Default run (a few minutes): synthetic undirected R-MAT graphs,
(a,b,c,d) = (0.57,0.19,0.19,0.05), int32 ids, int64 offsets, FP64 p and r,
optimized push rule:

* plain22 (the line's `value`): 2^22 vertices, edge factor 16, 16 seeds
  drawn uniformly from vertices of degree >= 1, run one after another,
  alpha = 0.01, eps = 1e-7.  A step is those 16 queries, each a full
  PR-Nibble push followed by the sweep cut, graph resident in HBM, and the
  copy of every query's p and cluster (support in sweep order with p on it)
  to the host.  The same steps without the copies are reported beside it.
* c1_rmat16: 2^16 vertices, edge factor 8, seed = the smallest vertex of the
  largest component (vertex 0), alpha 0.01, eps 1e-7: the saturating query
  (the diffusion covers the whole component over ~118 rounds).
* batched22: the 2^22 graph, 256 seeds in one batch (256 slots), eps
  log-uniform in [1e-7, 1e-5], alpha in {0.01, 0.05}; a step is the batch.
  Run twice: with dense per-slot state and with compact per-query tables.
* serve24: 2^24 vertices, seeds drawn proportionally to degree, eps
  log-uniform in [1e-7, 1e-4], alpha = 0.01, continuous batching over 256
  slots (compact tables: admission by memory): the saturation rate (all
  queries queued at once), then Poisson arrivals at 0.25, 0.5, 0.75 and 0.9
  of it, each with a 1 s warm-up and 10^4 measured queries, p50/p99 latency
  including the copy of each result to the host.
* large26: 2^26 vertices, 1024 seeds (32 of them the top-degree hubs), eps
  log-uniform in [1e-8, 1e-6], compact tables; one warm-up pass, one timed
  pass with no per-kernel events.

Prints one JSON line.  The roofline object describes the edge-scatter
launches, timed with HIP events on the library's stream in an instrumented
replay of the timed steps.  The CPU baseline is the oracle timed on the host
on a bounded sample of the headline queries.
"""
from __future__ import annotations

import argparse
import hashlib
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


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "scatter_hbm_traffic_rmat22.md")
# The plain path's edge scatter: the scatter launch (one FP64 atomic per edge,
# or pass A of the binned scatter on large rounds) and k_bin_apply (pass B),
# timed together per round.
PLAIN_SCATTER = "k_scatter + k_bin_apply"


def measured_traffic(kernel, bin_min_edges=None):
    """Per-launch HBM traffic of `kernel` from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the counter
    reads for a device copy of known size), or None when the kernel's sources
    changed since the counters were taken, or when the record names the
    plain path's binning threshold it was taken at and the live run bins from
    another (bin_min_edges: the live threshold, -1 when no round can bin)."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            block = f.read().split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)[kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, IndexError, KeyError, ValueError):
        return None
    if "plain_bin_min_edges" in rec and rec["plain_bin_min_edges"] != bin_min_edges:
        return None
    return rec if h.hexdigest()[:16] == rec["source_sha256_16"] else None


def roofline(tm, kernel, counted=True, bin_min_edges=None):
    """Roofline of the scatter kernel from the instrumented replay; the
    counter-based traffic only where the counters were taken on this same
    workload (counted=False for the others) and, for the plain scatter, at
    the same binning threshold."""
    sc = tm["scatter"]
    by = SCATTER_B_PER_EDGE * sc["units"] + SCATTER_B_PER_ENTRY * sc["entries"]
    gbs = by / (sc["ms"] * 1e-3) / 1e9 if sc["ms"] > 0 else 0.0
    tr = measured_traffic(kernel, bin_min_edges) if counted else None
    return {
        "kernel": "%s (edgeMap UpdateNgh)" % kernel, "bound": "hbm", "achieved": gbs,
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
        "traffic": tr["traffic_bytes_per_launch"] if tr else None,
        "traffic_unit": "bytes per launch (FETCH_SIZE x %.3f + WRITE_SIZE x %.3f)" % (
            tr["fetch_factor"], tr["write_factor"]) if tr else None,
        "traffic_over_algorithmic": tr["traffic_over_algorithmic"] if tr else None,
        "bytes_model": "20 B per pushed edge + 24 B per pushed vertex",
        "algorithmic_bytes_per_launch": by / max(sc["launches"], 1),
        "launches": sc["launches"], "avg_launch_us": sc["ms"] * 1e3 / max(sc["launches"], 1),
        "edges_per_s": sc["units"] / (sc["ms"] * 1e-3) if sc["ms"] > 0 else 0.0,
    }


def timed_steps(ctx, step, steps, warmup, instrument=True):
    """Warm-up, then the timed steps with no per-kernel events (an event node
    between dependent kernels costs about as much as a short kernel), then
    the same steps again with HIP events around every kernel on the
    library's stream: the kernel durations of the roofline come from that
    instrumented replay."""
    import torch
    acc = {"edges": 0, "pushes": 0, "rounds": 0, "support": 0, "queries": 0, "bin_rounds": 0}
    for i in range(warmup):
        step([], dict(acc))
        log("  warmup step %d done" % i)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(lat, acc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("  timed steps done")
    if not instrument:
        return elapsed, lat, acc, None
    ctx.timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat_i = []
    for _ in range(steps):
        step(lat_i, dict(acc))
    torch.cuda.synchronize()
    tm = ctx.timing_get()
    ctx.timing(False)
    tm["instrumented_replay"] = {"elapsed_s": time.perf_counter() - t1,
                                 "p50_ms": pct(lat_i, 50) * 1e3 if lat_i else None}
    log("  instrumented replay done")
    return elapsed, lat, acc, tm


def account(acc, infos, ids, ctx, fetch=False):
    """Sum the query counters; fetch copies every result's p and cluster to
    the host (all of the step's results with one GPU round trip) before the
    release."""
    for qid, info in zip(ids, infos):
        acc["edges"] += info["edges"]
        acc["pushes"] += info["pushes"]
        acc["rounds"] += info["rounds"]
        acc["support"] += info["support"]
        acc["queries"] += 1
        acc["bin_rounds"] = acc.get("bin_rounds", 0) + info["bin_rounds"]
    if fetch:
        ctx.results(ids, release=True)
    else:
        for qid in ids:
            ctx.release(qid)


def bench_plain(plc, synth, g, steps, warmup, bin_min_edges=0):
    seeds = synth.uniform_seeds(g, 16, seed=2)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20),
                      bin_min_edges=bin_min_edges)
    hg = ctx.load_graph(g.off, g.nbr)
    tune = ctx.autotune(hg, seeds, 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
    log("  plain launch shapes: self %d, scatter %d, sweep %d workgroups, binned rounds from %d "
        "edges (%d tried)" % (tune["plain_self"], tune["plain_scatter"], tune["plain_sweep"],
                              tune["plain_bin_min_edges"], tune["candidates"]))
    sl = [int(s) for s in seeds]

    def step(lat, acc):
        # the 16 queries one after another in one call (each synchronous in
        # the library), then every query's p and cluster copied to the host;
        # a query's latency is the library's own wall time from its start to
        # its result on the device
        ids, infos = ctx.run(hg, sl, 0.01, 1e-7, flags=plc.PLC_QF_NO_RESIDUAL)
        lat.extend(i["host_ns"] * 1e-9 for i in infos)
        account(acc, infos, ids, ctx, fetch=True)

    def step_resident(lat, acc):
        ids, infos = ctx.run(hg, sl, 0.01, 1e-7)
        lat.extend(i["host_ns"] * 1e-9 for i in infos)
        account(acc, infos, ids, ctx)

    elapsed, lat, acc, tm = timed_steps(ctx, step, steps, warmup)
    el2, lat2, acc2, _ = timed_steps(ctx, step_resident, steps, 1, instrument=False)
    dev = []
    ids, infos = ctx.run(hg, sl, 0.01, 1e-7)
    dev = [i["device_ns"] * 1e-6 for i in infos]
    for q in ids:
        ctx.release(q)
    ctx.close()
    nq = acc["queries"]
    return {
        "seeds": seeds, "elapsed": elapsed, "edges_per_s": acc["edges"] / elapsed,
        "queries_per_s": nq / elapsed, "ms_per_step": elapsed * 1e3 / steps,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "what": "per query: the library's wall time from its start to its "
                               "result on the device (a query queued behind the previous "
                               "one of the same call starts when that one is known done)"},
        "device_ms": {"p50": pct(dev, 50), "p99": pct(dev, 99),
                      "what": "per query: device clock from its initialisation kernel to the "
                              "end of its sweep"},
        "result_copy": "p and the cluster of every query copied to the host inside the "
                       "timed steps, the step's 16 results with one GPU round trip "
                       "(plc_result_copy_many; PLC_QF_NO_RESIDUAL: r is not kept)",
        "without_result_copy": {"edges_per_s": acc2["edges"] / el2,
                                "queries_per_s": acc2["queries"] / el2,
                                "ms_per_step": el2 * 1e3 / steps},
        "per_query": {k: acc[k] / nq for k in ("edges", "pushes", "rounds", "support",
                                                 "bin_rounds")},
        "kernels": tm,
        "roofline": roofline(tm, PLAIN_SCATTER, bin_min_edges=tune["plain_bin_min_edges"]),
        "launch_shapes": {k: tune[k] for k in ("plain_self", "plain_scatter", "plain_sweep",
                                               "plain_bin_min_edges")},
    }


def bench_c1(plc, synth, reps=5):
    """The saturating plain query: R-MAT 2^16 (edge factor 8) from the smallest
    vertex of the largest component, alpha 0.01, eps 1e-7."""
    import torch
    g = synth.rmat(16, 8, seed=1)
    x = synth.largest_component_min_vertex(g)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    for _ in range(2):
        ids, _ = ctx.run(hg, [x], 0.01, 1e-7)
        ctx.release(ids[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = {"edges": 0, "pushes": 0, "rounds": 0, "support": 0, "queries": 0, "bin_rounds": 0}
    lat = []
    for _ in range(reps):
        ids, infos = ctx.run(hg, [x], 0.01, 1e-7, flags=plc.PLC_QF_NO_RESIDUAL)
        lat.append(infos[0]["host_ns"] * 1e-9)
        account(acc, infos, ids, ctx, fetch=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = infos[0]
    ctx.close()
    return {"workload": "rmat16_ef8_plain_seed%d" % x, "n": g.n, "arcs": g.arcs, "seed": x,
            "alpha": 0.01, "eps": 1e-7, "queries": reps,
            "seconds_per_query": el / reps, "queries_per_s": reps / el,
            "edges_per_s": acc["edges"] / el,
            "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3},
            "per_query": {"edges": last["edges"], "pushes": last["pushes"],
                          "rounds": last["rounds"], "support": last["support"],
                          "bin_rounds": last["bin_rounds"], "bin_edges": last["bin_edges"],
                          "kstar": last["kstar"], "phi": last["phi"]}}


def bench_batched(plc, synth, g, steps, warmup, slots=256, compact=False):
    qs = synth.batched_queries(g, 256, seed=2, eps_lo=1e-7, eps_hi=1e-5)
    tables = (8 << 30) if compact else 0
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=compact,
                                              table_bytes=tables) + (512 << 20),
                      compact=compact)
    hg = ctx.load_graph(g.off, g.nbr)
    got = ctx.batch_reserve(hg, slots)
    tune = ctx.autotune(hg, qs.seeds, qs.alpha, qs.eps, plc.PLC_TUNE_BATCH)
    log("  batched launch shapes: self %d, scatter %d workgroups (%d tried)" % (
        tune["batch_self"], tune["batch_scatter"], tune["candidates"]))

    def step(lat, acc):
        # the batch in one call, then every query's p and cluster copied to
        # the host (the batch's results with one GPU round trip); the batch's
        # latency ends when its results are on the host
        q0 = time.perf_counter()
        ids, infos = ctx.run_batched(hg, qs.seeds, qs.alpha, qs.eps, flags=plc.PLC_QF_NO_RESIDUAL)
        account(acc, infos, ids, ctx, fetch=True)
        lat.append(time.perf_counter() - q0)

    def step_resident(lat, acc):
        ids, infos = ctx.run_batched(hg, qs.seeds, qs.alpha, qs.eps)
        account(acc, infos, ids, ctx)

    elapsed, lat, acc, tm = timed_steps(ctx, step, steps, warmup)
    el2, _, acc2, _ = timed_steps(ctx, step_resident, steps, 1, instrument=False)
    ctx.close()
    nq = acc["queries"]
    return {
        "queries": qs, "workload": "rmat%d_ef16_batched_256seeds" % (g.n.bit_length() - 1),
        "state": "compact tables" if compact else "dense slots", "slots": got, "edges_per_s": acc["edges"] / elapsed, "queries_per_s": nq / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "what": "per batch of 256, until its results are on the host"},
        "result_copy": "p and the cluster of every query copied to the host inside the "
                       "timed steps, the batch's 256 results with one GPU round trip "
                       "(plc_result_copy_many; PLC_QF_NO_RESIDUAL: r is not kept)",
        "without_result_copy": {"edges_per_s": acc2["edges"] / el2,
                                "queries_per_s": acc2["queries"] / el2,
                                "ms_per_step": el2 * 1e3 / steps,
                                "what": "the residual kept on the device, nothing copied"},
        "per_query": {k: acc[k] / nq for k in ("edges", "pushes", "rounds", "support")},
        "eps": [float(qs.eps.min()), float(qs.eps.max())], "alpha": [0.01, 0.05],
        "kernels": tm,
        "roofline": roofline(tm, "k_b_scatter<%s>" % ("CompactState" if compact else "DenseState")),
        "launch_shapes": {k: tune[k] for k in ("batch_self", "batch_scatter", "batch_sweep")},
    }


def bench_serving(plc, synth, scale, nq, slots=64, compact=False, measured=10000,
                  warmup_s=1.0, fracs=(0.25, 0.5, 0.75, 0.9)):
    import numpy as np
    from paper_1604_07515_amd import serve
    t0 = time.time()
    g = synth.rmat(scale, 16, seed=1)
    log("serving graph 2^%d: n=%d arcs=%d (%.1fs)" % (scale, g.n, g.arcs, time.time() - t0))
    rng = np.random.default_rng(2)
    pool = max(nq, 4 * measured)
    seeds = synth.degree_weighted_seeds(g, pool, rng)
    eps = 10.0 ** rng.uniform(-7, -4, pool)
    tables = (8 << 30) if compact else 0
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=compact,
                                              table_bytes=tables) + (1 << 30),
                      compact=compact)
    hg = ctx.load_graph(g.off, g.nbr)
    got = ctx.batch_reserve(hg, slots)
    ctx.autotune(hg, seeds[:128], 0.01, eps[:128], plc.PLC_TUNE_BATCH)
    flags = plc.PLC_QF_NO_RESIDUAL
    serve.serve(ctx, hg, seeds[:256], 0.01, eps[:256], np.zeros(256), fetch=True,
                flags=flags)  # warm-up
    sat = serve.serve(ctx, hg, seeds[:nq], 0.01, eps[:nq], np.zeros(nq), fetch=True, flags=flags)
    out = {"workload": "rmat%d_ef16_serving_poisson" % scale, "n": g.n, "arcs": g.arcs,
           "state": "compact tables" if compact else "dense slots", "slots": got,
           "alpha": 0.01, "eps": [1e-7, 1e-4], "seeds": "proportional to degree",
           "result_copy": "each result's p and cluster copied to the host before it counts "
                          "as done, the results of one engine step with one GPU round trip "
                          "(plc_result_copy_many; PLC_QF_NO_RESIDUAL)",
           "saturation": {"queries": nq, "queries_per_s": sat.queries_per_s,
                          "edges_per_s": sat.edges / sat.wall_s,
                          "p50_ms": sat.percentile_ms(50), "p99_ms": sat.percentile_ms(99)},
           "poisson": []}
    log("  saturation %.0f qps" % sat.queries_per_s)
    off = nq
    for frac in fracs:
        qps = frac * sat.queries_per_s
        k = int(qps * warmup_s) + measured
        idx = np.arange(off, off + k) % pool
        off += k
        arr = serve.poisson_arrivals(k, qps, np.random.default_rng(3))
        rep = serve.serve(ctx, hg, seeds[idx], 0.01, eps[idx], arr, warmup_s=warmup_s, fetch=True,
                          flags=flags)
        out["poisson"].append({"load": frac, "offered_qps": qps, "served_qps": rep.queries_per_s,
                               "measured_queries": int(len(rep.latency_s)),
                               "warmup_queries": rep.warmup_queries, "warmup_s": warmup_s,
                               "p50_ms": rep.percentile_ms(50), "p99_ms": rep.percentile_ms(99),
                               "max_in_flight": rep.max_in_flight})
        log("  poisson %.2f x saturation (%.0f qps): p50 %.2f ms p99 %.2f ms, %d measured" % (
            frac, qps, rep.percentile_ms(50), rep.percentile_ms(99), len(rep.latency_s)))
    ctx.close()
    return out


def bench_large(plc, synth, scale=26, nq=1024, slots=1024, table_gib=160):
    """1024 seeds (32 of them the top-degree hubs) on R-MAT 2^scale with eps
    log-uniform in [1e-8, 1e-6], alpha 0.01, through the compact-table engine:
    queries are admitted as table memory allows.  Driven step by step (so that
    progress is printed); each result is released as soon as it is read."""
    import numpy as np
    t0 = time.time()
    g = synth.rmat(scale, 16, seed=1)
    log("large graph 2^%d: n=%d arcs=%d maxdeg=%d (%.1fs)" % (scale, g.n, g.arcs, g.deg.max(),
                                                             time.time() - t0))
    hubs = np.argsort(-g.deg, kind="stable")[:32]
    seeds = np.concatenate([synth.uniform_seeds(g, nq - 32, seed=2), hubs])
    eps = 10.0 ** np.random.default_rng(2).uniform(-8, -6, nq)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=True,
                                              table_bytes=table_gib << 30), compact=True)
    hg = ctx.load_graph(g.off, g.nbr)
    got = ctx.batch_reserve(hg, slots)
    import torch

    def one_pass(tag):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ids = ctx.submit(hg, seeds, 0.01, eps)
        done, acc, last_log = 0, {"edges": 0, "support": 0, "rounds": 0, "nomem": 0}, t1
        left = len(ids)
        while left > 0:
            fin = []
            left = ctx.progress(hg, fin)
            for qid in fin:
                info = ctx.result_info(qid)
                if info["status"] == plc.PLC_E_NOMEM:
                    acc["nomem"] += 1
                acc["edges"] += info["edges"]
                acc["support"] = max(acc["support"], info["support"])
                acc["rounds"] = max(acc["rounds"], info["rounds"])
                ctx.release(qid)
                done += 1
            if time.perf_counter() - last_log > 10:
                last_log = time.perf_counter()
                log("  large %s: %d of %d done (%.0fs)" % (tag, done, nq, last_log - t1))
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        log("  large %s pass: %.2f s" % (tag, el))
        return el, acc

    one_pass("warm-up")
    elapsed, acc = one_pass("timed")
    ctx.timing(True)
    el_i, _ = one_pass("instrumented")
    tm = ctx.timing_get()
    ctx.timing(False)
    # a sweep at this scale: Nibble (T = 2, nothing truncated) from the top
    # hub covers every vertex within two hops of it (one warm run, one timed
    # run, one with the sweep's events on)
    hub = int(hubs[0])
    qid, _ = ctx.run_nibble(hg, hub, 1e-300, 2)
    ctx.release(qid)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    qid, hinfo = ctx.run_nibble(hg, hub, 1e-300, 2)
    el_h = time.perf_counter() - t2
    ctx.release(qid)
    ctx.timing(True)
    qid, _ = ctx.run_nibble(hg, hub, 1e-300, 2)
    ctx.release(qid)
    th = ctx.timing_get()
    ctx.timing(False)
    ctx.close()
    hub_sweep = {"query": "Nibble, T 2, eps 1e-300, from the top hub (vertex %d)" % hub,
                 "support": hinfo["support"], "kstar": hinfo["kstar"],
                 "pushed_edges": hinfo["edges"], "ms": el_h * 1e3,
                 "sweep_ms": th["sweep"]["ms"], "sweep_support_arcs": th["sweep"]["units"]}
    log("  large hub sweep: support %d in %.1f ms (sweep %.1f ms)" % (
        hinfo["support"], el_h * 1e3, th["sweep"]["ms"]))
    return {"workload": "rmat%d_ef16_1024seeds_32hubs" % scale, "n": g.n, "arcs": g.arcs,
            "state": "compact tables", "slots": got, "table_budget_gib": table_gib,
            "eps": [1e-8, 1e-6], "alpha": 0.01, "queries": nq, "failed_nomem": acc["nomem"],
            "elapsed_s": elapsed, "edges_per_s": acc["edges"] / elapsed,
            "queries_per_s": nq / elapsed, "max_support": acc["support"],
            "max_rounds": acc["rounds"], "kernels": tm,
            "what": "one warm-up pass, then the timed pass (no per-kernel events), then an "
                    "instrumented pass for the kernel durations (%.2f s)" % el_i,
            "roofline": roofline(tm, "k_b_scatter<CompactState>", counted=False),
            "hub_sweep": hub_sweep}


def bench_rules(plc, synth, g, seeds):
    """The paper's comparison of the two push rules (Sec. 3.3, "An
    Optimization": the optimized rule reaches the same conductance with less
    work): the 16 plain seeds under each rule, one warm pass, then one timed
    pass each."""
    import numpy as np
    import torch
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    ctx.autotune(hg, seeds[:4], 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
    out = {}
    for name, rule in (("optimized", plc.PLC_RULE_OPT), ("original", plc.PLC_RULE_ORIG)):
        for timed in (False, True):
            rows = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for x in seeds:
                ids, infos = ctx.run(hg, [int(x)], 0.01, 1e-7, rule)
                ctx.release(ids[0])
                rows.append(infos[0])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        out[name] = {"ms_per_query": el * 1e3 / len(seeds),
                     "pushes_per_query": float(np.mean([r["pushes"] for r in rows])),
                     "edges_per_query": float(np.mean([r["edges"] for r in rows])),
                     "rounds_per_query": float(np.mean([r["rounds"] for r in rows])),
                     "phi": [r["phi"] for r in rows]}
    # the beta variant (end of Sec. 3.3): only the top fraction of the active
    # set by r/d is pushed per round (rounds launched directly)
    for beta in (0.5, 0.25):
        for timed in (False, True):
            rows = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for x in seeds:
                qid, info = ctx.run_beta(hg, int(x), 0.01, 1e-7, beta)
                ctx.release(qid)
                rows.append(info)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        out["beta_%g" % beta] = {"ms_per_query": el * 1e3 / len(seeds),
                                  "pushes_per_query": float(np.mean([r["pushes"] for r in rows])),
                                  "rounds_per_query": float(np.mean([r["rounds"] for r in rows])),
                                  "phi": [r["phi"] for r in rows]}
    ctx.close()
    po, pr = np.array(out["optimized"]["phi"]), np.array(out["original"]["phi"])
    return {"workload": "rmat22_ef16_plain_16seeds", "alpha": 0.01, "eps": 1e-7,
            "optimized": {k: v for k, v in out["optimized"].items() if k != "phi"},
            "original": {k: v for k, v in out["original"].items() if k != "phi"},
            "speedup_optimized": out["original"]["ms_per_query"] / out["optimized"]["ms_per_query"],
            "push_ratio": out["original"]["pushes_per_query"] / out["optimized"]["pushes_per_query"],
            "phi_optimized_over_original": {"median": float(np.median(po / pr)),
                                            "min": float(np.min(po / pr)),
                                            "max": float(np.max(po / pr))},
            "paper": "sequential, optimized rule 1.4-6.4x faster at the same conductance",
            "beta": {("%g" % b): {"ms_per_query": out["beta_%g" % b]["ms_per_query"],
                                  "pushes_per_query": out["beta_%g" % b]["pushes_per_query"],
                                  "rounds_per_query": out["beta_%g" % b]["rounds_per_query"],
                                  "phi_median_over_beta1": float(np.median(
                                      np.array(out["beta_%g" % b]["phi"]) / po))}
                     for b in (0.5, 0.25)}}


def algo_timed(run, seeds, params):
    """One query at a time through `run(seed) -> (id, info)` (which releases
    its result): one warm pass over the seeds, then one timed pass."""
    import numpy as np
    import torch
    for timed in (False, True):
        rows = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for x in seeds:
            qid, info = run(int(x))
            rows.append((qid, info))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    infos = [r for _, r in rows]
    nq = len(seeds)
    edges = sum(r["edges"] for r in infos)
    out = dict(params)
    out.update({"queries": nq, "seconds_per_query": el / nq, "queries_per_s": nq / el,
                "edges_per_s": edges / el,
                "per_query": {"rounds": float(np.mean([r["rounds"] for r in infos])),
                              "pushes": float(np.mean([r["pushes"] for r in infos])),
                              "edges": edges / nq,
                              "support": float(np.mean([r["support"] for r in infos]))}})
    return out


def hkpr_timed(ctx, hg, seeds, N=20, eps=1e-7, t=10.0):
    """Deterministic HK-PR + sweep (Sec. 3.4) with the paper's experiment
    parameters (t = 10, N = 20, eps = 1e-7)."""
    def run(x):
        qid, info = ctx.run_hkpr(hg, x, N, eps, t)
        ctx.release(qid)
        return qid, info
    return algo_timed(run, seeds, {"algorithm": "HK-PR", "N": N, "eps": eps, "t": t})


def nibble_timed(ctx, hg, seeds, T=20, eps=1e-8):
    """Nibble + sweep (Sec. 3.2) with the paper's experiment parameters
    (T = 20, eps = 1e-8)."""
    def run(x):
        qid, info = ctx.run_nibble(hg, x, eps, T)
        ctx.release(qid)
        return qid, info
    return algo_timed(run, seeds, {"algorithm": "Nibble", "T": T, "eps": eps})


def bench_hkpr(plc, synth, g, seeds):
    """HK-PR and Nibble with the paper's parameters on the 16 plain seeds."""
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    ctx.autotune(hg, seeds[:4], 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
    out = hkpr_timed(ctx, hg, seeds)
    out["workload"] = "rmat22_ef16_hkpr_16seeds"
    nb = nibble_timed(ctx, hg, seeds)
    nb["workload"] = "rmat22_ef16_nibble_16seeds"
    ctx.close()
    return out, nb


def one_at_a_time(plc, g, seeds, alpha=0.01, eps=1e-7):
    """Plain PR-Nibble + sweep queries on g one at a time (each its own
    plc_run call, timed from the host), after an autotune and two warm
    queries.  Returns the open context, the graph handle and the figures."""
    import torch
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20))
    hg = ctx.load_graph(g.off, g.nbr)
    tune = ctx.autotune(hg, seeds[:2], alpha, eps, plc.PLC_TUNE_PLAIN)
    for s in seeds[:2]:
        ids, _ = ctx.run(hg, [s], alpha, eps)
        ctx.release(ids[0])
    lat, acc = [], {"edges": 0, "pushes": 0, "rounds": 0, "support": 0, "queries": 0}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in seeds:
        q0 = time.perf_counter()
        ids, infos = ctx.run(hg, [s], alpha, eps)
        lat.append(time.perf_counter() - q0)
        account(acc, infos, ids, ctx)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    nq = len(seeds)
    per = el / nq
    return ctx, hg, {"n": g.n, "arcs": g.arcs, "alpha": alpha, "eps": eps, "queries": nq,
                     "seconds_per_query": per, "queries_per_s": nq / el,
                     "edges_per_s": acc["edges"] / el,
                     "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3},
                     "per_query": {k: acc[k] / nq for k in ("edges", "pushes", "rounds",
                                                            "support")},
                     "bin_min_edges": tune["plain_bin_min_edges"]}


def bench_grid3d(plc, synth, side=215, nq=8):
    """The paper's 3D-grid input (a side^3 torus, every vertex of degree 6;
    side 215 gives its n = 9,938,375 and 3n edges): one PR-Nibble + sweep at a
    time, alpha 0.01, eps 1e-7, optimized rule, as in the paper's PR-Nibble
    timing (40 cores: 0.502 s per query).  Every vertex of a torus is
    equivalent, so the seeds only relabel the same query."""
    import numpy as np
    t0 = time.time()
    g = synth.torus3d(side)
    log("grid3d %d^3: n=%d arcs=%d (%.1fs)" % (side, g.n, g.arcs, time.time() - t0))
    seeds = [int(x) for x in np.random.default_rng(3).integers(0, g.n, nq)]
    ctx, hg, out = one_at_a_time(plc, g, seeds)
    hk = hkpr_timed(ctx, hg, seeds)
    nb = nibble_timed(ctx, hg, seeds)
    ctx.close()
    hk["paper_40core_seconds_per_query"] = 0.049
    hk["paper_1thread_seconds_per_query"] = 0.01
    nb["paper_40core_seconds_per_query"] = 0.040
    nb["paper_1thread_seconds_per_query"] = 0.01
    out.update({"workload": "torus%d_3dgrid_plain" % side, "hkpr": hk, "nibble": nb,
                "paper_40core_seconds_per_query": 0.502,
                "speedup_vs_paper_40core": 0.502 / out["seconds_per_query"]})
    return out


def randlocal_batched(plc, synth, g, nq=256, table_gib=64):
    """nq queries at once (same setting as the plain leg, seeds uniform over
    all vertices) through the compact-table engine, one slot per query; one
    warm batch of 16, then the timed batch."""
    import torch
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, nq, compact=True,
                                              table_bytes=table_gib << 30), compact=True)
    hg = ctx.load_graph(g.off, g.nbr)
    assert ctx.batch_reserve(hg, nq) == nq
    ids, _ = ctx.run_batched(hg, [int(x) for x in synth.uniform_seeds(g, 16, seed=4)],
                             0.01, 1e-7)
    for q in ids:
        ctx.release(q)
    seeds = [int(x) for x in synth.uniform_seeds(g, nq, seed=2)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ids, infos = ctx.run_batched(hg, seeds, 0.01, 1e-7)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    edges = sum(int(i["edges"]) for i in infos)
    for q in ids:
        ctx.release(q)
    ctx.close()
    return {"queries": nq, "slots": nq, "seconds": el, "queries_per_s": nq / el,
            "edges_per_s": edges / el, "per_query_edges": edges / nq}


def bench_randlocal(plc, synth, n=10_000_000, nq=8):
    """The paper's randLocal input at its size (n = 10^7, five drawn
    neighbours per vertex, offsets favouring near ids; 49.1 M distinct edges):
    one PR-Nibble + sweep at a time, alpha 0.01, eps 1e-7, optimized rule,
    seeds uniform over all vertices (every vertex has degree >= 2), against
    the paper's PR-Nibble timing on it (40 cores: 1.250 s per query; one
    thread 28.90 s)."""
    t0 = time.time()
    g = synth.rand_local(n)
    log("randlocal n=%d: arcs=%d (%.1fs)" % (g.n, g.arcs, time.time() - t0))
    seeds = [int(x) for x in synth.uniform_seeds(g, nq, seed=2)]
    ctx, hg, out = one_at_a_time(plc, g, seeds)
    ctx.close()
    out["batched_compact"] = randlocal_batched(plc, synth, g)
    out.update({"workload": "randlocal%d_k5_plain" % n,
                "paper_40core_seconds_per_query": 1.250,
                "paper_1thread_seconds_per_query": 28.90,
                "speedup_vs_paper_40core": 1.250 / out["seconds_per_query"]})
    return out


def cpu_baseline(oracle, g, work, budget, what):
    """The oracle, single-threaded, on the given queries in order (the list
    repeated until `budget` seconds of work)."""
    c0 = time.perf_counter()
    done = e_sum = 0
    while work and time.perf_counter() - c0 <= budget:
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
            "sample": "%d queries: %s; single-threaded oracle push + sweep on the same "
                      "R-MAT 2^22 graph, %.1f s" % (done, what, ct)}


def cpu_multicore_baseline(g, work, budget):
    """The OpenMP PR-Nibble + sweep (all host threads) on the same queries in
    the same order, repeated until `budget` seconds."""
    import cpu_multicore
    s = cpu_multicore.Solver(g.off, g.nbr)
    try:
        c0 = time.perf_counter()
        done = e_sum = 0
        while work and time.perf_counter() - c0 <= budget:
            for sd, al, ep in work:
                e_sum += s.run(int(sd), float(al), float(ep))["edges"]
                done += 1
                if time.perf_counter() - c0 > budget:
                    break
        ct = time.perf_counter() - c0
    finally:
        s.close()
    return {"value": e_sum / ct, "unit": "pushed edges/s", "cores": cpu_multicore.threads(),
            "kind": "openmp", "queries_per_s": done / ct,
            "sample": "%d queries (the headline's 16 plain queries in order, repeated), OpenMP "
                      "push with atomic adds + parallel sweep, %.1f s" % (done, ct)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--only", choices=["plain", "c1", "batched", "serving", "large", "grid3d",
                                       "randlocal"],
                    default=None,
                    help="run one workload only (the others are reported as skipped)")
    ap.add_argument("--skip", action="append", default=[],
                    choices=["c1", "batched", "serving", "large", "grid3d", "randlocal"],
                    help="leave a workload out of the default run")
    ap.add_argument("--serve-measured", type=int, default=10000,
                    help="measured queries per Poisson load (after a 1 s warm-up)")
    ap.add_argument("--serve-scale", type=int, default=24)
    ap.add_argument("--serve-queries", type=int, default=2048)
    ap.add_argument("--serve-state", choices=["dense", "compact"], default="compact",
                    help="state layout of the serving engine")
    ap.add_argument("--serve-slots", type=int, default=256,
                    help="batch slots of the serving engine")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline on the headline "
                         "queries (0 = skip)")
    ap.add_argument("--cpu-mix-budget", type=float, default=5.0,
                    help="seconds of oracle time on the plain and batched queries together "
                         "(0 = skip)")
    ap.add_argument("--cpu-mc-budget", type=float, default=10.0,
                    help="seconds for the multicore (OpenMP) CPU baseline (0 = skip)")
    ap.add_argument("--plain-bin-min-edges", type=int, default=0, metavar="EDGES",
                    help="the plain leg's binning threshold: 0 = picked by the autotuner "
                         "(default), > 0 = rounds of at least EDGES edges binned, < 0 = none "
                         "(fixes the configuration for hardware-counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a device copy of MIB MiB three times (reference kernel "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(seeds would shard across GPUs, one graph replica each); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import synth
    import paper_1604_07515_amd as plc

    if args.copy_calibration > 0:
        import torch
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x %d MiB device copies" % args.copy_calibration)
        del src, dst

    t0 = time.time()
    g = synth.rmat(22, 16, seed=1)
    log("graph 2^22: n=%d arcs=%d maxdeg=%d (%.1fs)" % (g.n, g.arcs, g.deg.max(), time.time() - t0))
    want = lambda w: (args.only is None and w not in args.skip) or args.only == w
    plain = (bench_plain(plc, synth, g, args.steps, args.warmup, args.plain_bin_min_edges)
             if want("plain") else None)
    if plain:
        log("plain: %.3g edges/s, %.1f queries/s" % (plain["edges_per_s"], plain["queries_per_s"]))
    c1 = bench_c1(plc, synth) if want("c1") else None
    if c1:
        log("c1 (R-MAT 2^16 from vertex %d): %.2f ms per query, %.3g edges/s, %d rounds, "
            "%d binned" % (c1["seed"], c1["seconds_per_query"] * 1e3, c1["edges_per_s"],
                           c1["per_query"]["rounds"], c1["per_query"]["bin_rounds"]))
    bat = bench_batched(plc, synth, g, max(3, args.steps // 2), 2) if want("batched") else None
    if bat:
        log("batched: %.3g edges/s, %.1f queries/s" % (bat["edges_per_s"], bat["queries_per_s"]))
    bat_c = (bench_batched(plc, synth, g, max(3, args.steps // 2), 2, compact=True)
             if want("batched") else None)
    if bat_c:
        log("batched (compact tables): %.3g edges/s, %.1f queries/s" % (
            bat_c["edges_per_s"], bat_c["queries_per_s"]))
    srv = (bench_serving(plc, synth, args.serve_scale, args.serve_queries, args.serve_slots,
                         compact=args.serve_state == "compact", measured=args.serve_measured)
           if want("serving") else None)
    rules = bench_rules(plc, synth, g, plain["seeds"]) if plain else None
    if rules:
        log("rules: optimized %.2f ms/query, original %.2f ms/query (%.2fx), pushes x%.2f" % (
            rules["optimized"]["ms_per_query"], rules["original"]["ms_per_query"],
            rules["speedup_optimized"], rules["push_ratio"]))
    hkpr, nibble = bench_hkpr(plc, synth, g, plain["seeds"]) if plain else (None, None)
    if hkpr:
        log("hkpr: %.2f ms/query, %.3g edges/s; nibble: %.2f ms/query, %.3g edges/s" % (
            hkpr["seconds_per_query"] * 1e3, hkpr["edges_per_s"],
            nibble["seconds_per_query"] * 1e3, nibble["edges_per_s"]))
    grid = bench_grid3d(plc, synth) if want("grid3d") else None
    if grid:
        log("grid3d: %.2f ms per query (%.0fx the paper's 40-core time); HK-PR %.2f ms; "
            "Nibble %.2f ms" % (grid["seconds_per_query"] * 1e3, grid["speedup_vs_paper_40core"],
                                grid["hkpr"]["seconds_per_query"] * 1e3,
                                grid["nibble"]["seconds_per_query"] * 1e3))
    rloc = bench_randlocal(plc, synth) if want("randlocal") else None
    if rloc:
        log("randlocal: %.2f ms per query (%.0fx the paper's 40-core time), %.3g edges/s; "
            "batched (compact): %.1f queries/s, %.3g edges/s" % (
                rloc["seconds_per_query"] * 1e3, rloc["speedup_vs_paper_40core"],
                rloc["edges_per_s"], rloc["batched_compact"]["queries_per_s"],
                rloc["batched_compact"]["edges_per_s"]))
    big = bench_large(plc, synth) if want("large") else None
    if big:
        log("large: %.3g edges/s, %.1f queries/s" % (big["edges_per_s"], big["queries_per_s"]))

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
                   {"workload": bat["workload"], "n": g.n, "arcs": g.arcs} if bat else
                   {"workload": (srv or big or grid or rloc or {}).get("workload")}),
    }
    if main_res:
        out["queries_per_s"] = main_res["queries_per_s"]
        out["latency_ms"] = main_res["latency_ms"]
        out["per_query"] = main_res["per_query"]
        out["roofline"] = main_res["roofline"]
        out["kernels"] = main_res["kernels"]
        for k in ("device_ms", "result_copy", "without_result_copy"):
            if k in main_res:
                out[k] = main_res[k]
        out["launch_shapes"] = main_res["launch_shapes"]
    if bat:
        out["batched"] = {k: v for k, v in bat.items() if k != "queries"}
        if plain:
            out["batched"]["queries_per_s_vs_plain"] = bat["queries_per_s"] / plain["queries_per_s"]
    if bat_c:
        out["batched_compact"] = {k: v for k, v in bat_c.items() if k != "queries"}
    if big:
        out["large"] = big
    if c1:
        out["c1"] = c1
    if grid:
        out["grid3d"] = grid
    if rloc:
        out["randlocal"] = rloc
    if rules:
        out["rules"] = rules
    if hkpr:
        out["hkpr"] = hkpr
        out["nibble"] = nibble
    if srv:
        out["serving"] = srv
    head = [(s, 0.01, 1e-7) for s in plain["seeds"]] if plain else []
    mix = list(head)
    if bat:
        q = bat["queries"]
        mix += list(zip(q.seeds, q.alpha, q.eps))
    if args.cpu_budget > 0 and head:
        import oracle
        out["cpu_baseline"] = cpu_baseline(
            oracle, g, head, args.cpu_budget,
            "the headline workload: the 16 plain R-MAT 2^22 queries (alpha 0.01, eps 1e-7) in "
            "order, repeated")
    if args.cpu_mix_budget > 0 and mix:
        import oracle
        out["cpu_baseline_mix"] = cpu_baseline(
            oracle, g, mix, args.cpu_mix_budget,
            "the 16 plain queries, then the 256 batched queries, in order, repeated")
    if args.cpu_mc_budget > 0 and head:
        out["cpu_multicore"] = cpu_multicore_baseline(g, head, args.cpu_mc_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
