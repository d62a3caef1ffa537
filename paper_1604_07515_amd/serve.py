"""Continuous-batching request loop over a libplc batch engine.

Queries arrive at given times (e.g. a Poisson process).  Every arrival is
submitted as soon as the wall clock passes its arrival time; each
``plc_progress`` step then admits queued queries into the slots freed by
retiring ones, runs one PR-Nibble round for every admitted query in the same
launches and sweeps the queries that finished pushing.  Queries that arrive
while others run therefore join the running batch at the next round
boundary.  Latency of a query = time its result became available - its
arrival time.

The loop is host orchestration only (clock, bookkeeping); all clustering
work runs in libplc's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServeReport:
    latency_s: np.ndarray          # per measured query, in arrival order
    ids: np.ndarray                # query handles (results kept until released)
    wall_s: float                  # measured window: first measured arrival to last completion
    steps: int                     # plc_progress calls
    busy_steps: int = 0
    max_in_flight: int = 0
    edges: int = 0
    warmup_queries: int = 0        # arrivals inside the warm-up window (not measured)
    extra: dict = field(default_factory=dict)

    @property
    def queries_per_s(self) -> float:
        return len(self.latency_s) / self.wall_s if self.wall_s > 0 else 0.0

    def percentile_ms(self, q: float) -> float:
        return float(np.percentile(self.latency_s, q) * 1e3)


def poisson_arrivals(count: int, qps: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    if qps <= 0 or not np.isfinite(qps):
        return np.zeros(count)
    return np.cumsum(rng.exponential(1.0 / qps, count))


def serve(ctx, g, seeds, alphas, epss, arrivals, release: bool = True,
          clock=time.perf_counter, warmup_s: float = 0.0, fetch: bool = False,
          flags: int = 0) -> ServeReport:
    """Run the request loop until every query has finished.

    seeds, alphas, epss: per-query parameters; arrivals: non-decreasing
    arrival times in seconds from the start of the loop.  Queries arriving
    before warmup_s run but are left out of the latencies and the rate.
    fetch: copy each finished query's result (support in sweep order and p
    on it, so the cluster and p) to the host before it counts as done.
    """
    seeds = np.asarray(seeds)
    alphas = np.broadcast_to(np.asarray(alphas, np.float64), seeds.shape)
    epss = np.broadcast_to(np.asarray(epss, np.float64), seeds.shape)
    arrivals = np.asarray(arrivals, np.float64)
    n = len(seeds)
    lat = np.full(n, np.nan)
    ids = np.zeros(n, np.uint64)
    index = {}
    nxt = 0
    steps = busy = max_fl = 0
    edges = 0
    t0 = clock()
    while nxt < n or index:
        now = clock() - t0
        j = int(np.searchsorted(arrivals, now, side="right"))
        if j > nxt:
            new = ctx.submit(g, seeds[nxt:j], alphas[nxt:j], epss[nxt:j], flags=flags)
            for k, qid in enumerate(new):
                index[qid] = nxt + k
                ids[nxt + k] = qid
            nxt = j
        if index:
            done = []
            left = ctx.progress(g, done)
            steps += 1
            busy += 1
            max_fl = max(max_fl, left + len(done))
            if fetch and done:
                # every result the step finished, copied with one GPU round trip
                for res in ctx.results(done, release=release):
                    edges += res.info["edges"]
            for qid in done:
                i = index.pop(qid)
                if not fetch and release:
                    info = ctx.result_info(qid)
                    edges += info["edges"]
                    ctx.release(qid)
                lat[i] = (clock() - t0) - arrivals[i]
        elif nxt < n:
            wait = arrivals[nxt] - (clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    end = clock() - t0
    meas = arrivals >= warmup_s if warmup_s > 0 else np.ones(n, bool)
    first = arrivals[meas][0] if meas.any() else 0.0
    wall = end - first
    return ServeReport(lat[meas], ids, wall, steps, busy, max_fl, edges,
                       warmup_queries=int(n - meas.sum()))


def saturation(ctx, g, seeds, alphas, epss) -> ServeReport:
    """Closed loop: every query available at time 0 (the engine's peak rate)."""
    return serve(ctx, g, seeds, alphas, epss, np.zeros(len(seeds)))
