"""Parity at the benchmark's full sizes, in the launch shapes it times.

* plain: R-MAT 2^22 (ef 16), the benchmark's 16 uniform seeds, alpha 0.01,
  eps 1e-7, after the same autotuning; every query against the oracle.
* batched: the same graph, the benchmark's 256 queries (eps log-uniform in
  [1e-7, 1e-5], alpha in {0.01, 0.05}) through 256 slots after autotuning;
  a sample of 64 against the oracle, properties that hold at any size
  (mass, termination, the reported cut and volume recounted from the
  cluster) on all 256.
* serving: R-MAT 2^24, degree-weighted seeds, eps log-uniform in
  [1e-7, 1e-4], 64 slots, Poisson arrivals; a sample against the oracle,
  properties on all, and a few queries re-run alone.
"""
import sys

import numpy as np
import pytest

import synth
from parity import check_properties, check_query, check_same

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def plc():
    import paper_1604_07515_amd as plc
    return plc


@pytest.fixture(scope="module")
def g22():
    return synth.rmat(22, 16, seed=1)


def test_plain_rmat22_bench_shapes(plc, g22):
    g = g22
    seeds = synth.uniform_seeds(g, 16, seed=2)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        tune = ctx.autotune(hg, seeds, 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
        say("plain 2^22 shapes", tune["plain_self"], tune["plain_scatter"], tune["plain_sweep"])
        ids, infos = ctx.run(hg, seeds, 0.01, 1e-7)
        for i, qid in enumerate(ids):
            say("plain 2^22 seed", int(seeds[i]))
            check_query(g, ctx.result(qid, release=True), int(seeds[i]), 0.01, 1e-7, 0)
    finally:
        ctx.close()


def test_batched_rmat22_bench_shapes(plc, g22):
    g = g22
    qs = synth.batched_queries(g, 256, seed=2, eps_lo=1e-7, eps_hi=1e-5)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, 256) + (512 << 20))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 256) == 256
        tune = ctx.autotune(hg, qs.seeds, qs.alpha, qs.eps, plc.PLC_TUNE_BATCH)
        say("batched 2^22 shapes", tune["batch_self"], tune["batch_scatter"])
        ids, infos = ctx.run_batched(hg, qs.seeds, qs.alpha, qs.eps)
        sample = set(np.argsort(qs.eps)[::4].tolist())  # every 4th eps, smallest to largest
        for i, qid in enumerate(ids):
            res = ctx.result(qid, release=True)
            check_properties(g, res, float(qs.eps[i]))
            if i in sample:
                check_query(g, res, int(qs.seeds[i]), float(qs.alpha[i]), float(qs.eps[i]), 0)
        say("batched 2^22: %d checked against the oracle" % len(sample))
    finally:
        ctx.close()


def test_serving_rmat24_bench_shapes(plc):
    from paper_1604_07515_amd import serve
    g = synth.rmat(24, 16, seed=1)
    say("serving graph 2^24 arcs", g.arcs)
    rng = np.random.default_rng(2)
    nq = 256
    seeds = synth.degree_weighted_seeds(g, 2048, rng)[:nq]
    eps = (10.0 ** rng.uniform(-7, -4, 2048))[:nq]
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, 64) + (1 << 30))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 64) == 64
        ctx.autotune(hg, seeds[:128], 0.01, eps[:128], plc.PLC_TUNE_BATCH)
        arr = serve.poisson_arrivals(nq, 4000.0, np.random.default_rng(3))
        rep = serve.serve(ctx, hg, seeds, 0.01, eps, arr, release=False)
        say("serving 2^24: %.0f q/s, max in flight %d" % (rep.queries_per_s, rep.max_in_flight))
        assert rep.max_in_flight > 1
        results = [ctx.result(int(qid), release=True) for qid in rep.ids]
        for i, res in enumerate(results):
            check_properties(g, res, float(eps[i]))
        for i in range(0, nq, 8):
            say("serving 2^24 oracle query", i)
            check_query(g, results[i], int(seeds[i]), 0.01, float(eps[i]), 0)
        for i in (0, 101, 255):
            ids1, _ = ctx.run_batched(hg, [int(seeds[i])], 0.01, float(eps[i]))
            check_same(g, ctx.result(ids1[0], release=True), results[i])
    finally:
        ctx.close()
