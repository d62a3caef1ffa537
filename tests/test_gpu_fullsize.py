"""Parity at the benchmark's full sizes, in the launch shapes it times.

* plain: R-MAT 2^22 (ef 16), the benchmark's 16 uniform seeds, alpha 0.01,
  eps 1e-7, after the same autotuning, with the same query flags (no
  residual kept; p and the cluster copied back); every query against the
  oracle, and the same queries with the residual kept; then all again with
  the binning threshold fixed at its default.
* batched: the same graph, the benchmark's 256 queries (eps log-uniform in
  [1e-7, 1e-5], alpha in {0.01, 0.05}) through 256 slots after autotuning,
  with dense slots and with compact tables (8 GiB of tables, as timed); a
  sample of 64 against the oracle, properties that hold at any size (mass,
  termination, the reported cut and volume recounted from the cluster) on
  all 256.
* serving: R-MAT 2^24, degree-weighted seeds, eps log-uniform in
  [1e-7, 1e-4], compact tables over 256 slots and no residual kept, as the
  benchmark serves them, Poisson arrivals; a sample against the oracle,
  properties on all, and a few queries re-run alone.
* Nibble from the top hub of R-MAT 2^22 with T = 2 and no truncation: a
  support of 2,208,937 vertices (more than 2^21), so the sweep's deepest
  merge passes and multi-million scans are checked against the oracle.

Every oracle comparison is strict (p and r to 1e-12, counters, order,
cluster) unless the oracle reports a threshold decision within 1e-10 of its
threshold; for these inputs the oracle flags none, and the tests assert that
every sampled query was checked strictly.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import RTOL, check_nibble, check_properties, check_query, check_same

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


def strict_report(name, reports):
    """Print and return the number of strictly checked queries; the flagged
    ones are listed with the oracle's gap."""
    flagged = [(i, r["gap"]) for i, r in reports if r["tie_push"]]
    say("%s: %d of %d checked strictly; flagged (index, gap): %s" % (
        name, len(reports) - len(flagged), len(reports), flagged))
    return len(reports) - len(flagged)


def test_plain_rmat22_bench_shapes(plc, g22):
    """The benchmark's plain queries in its launch configuration (autotuned
    shapes and binning threshold), then again with the binning threshold
    fixed at its default so that the binned rounds are checked at full size
    whatever the tuner picked."""
    g = g22
    seeds = synth.uniform_seeds(g, 16, seed=2)
    sl = [int(s) for s in seeds]
    orcs = [oracle.prnibble(g.off, g.nbr, x, 0.01, 1e-7) for x in sl]
    for fixed in (0, 524288):
        ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20),
                          bin_min_edges=fixed)
        name = "plain 2^22 (%s)" % ("tuned" if fixed == 0 else "binned from 524288 edges")
        try:
            hg = ctx.load_graph(g.off, g.nbr)
            tune = ctx.autotune(hg, seeds, 0.01, 1e-7, plc.PLC_TUNE_PLAIN)
            say(name, "shapes", tune["plain_self"], tune["plain_scatter"], tune["plain_sweep"],
                "binning threshold", tune["plain_bin_min_edges"])
            ids, infos = ctx.run(hg, sl, 0.01, 1e-7, flags=plc.PLC_QF_NO_RESIDUAL)
            # the benchmark's copy: all 16 results in one call (several MiB,
            # so the host part is split among threads)
            many = ctx.results(ids, release=True)
            ids_r, _ = ctx.run(hg, sl, 0.01, 1e-7)
            reps = []
            for i, (res, qr) in enumerate(zip(many, ids_r)):
                say(name, "seed", sl[i], "binned rounds", infos[i]["bin_rounds"])
                reps.append((i, check_query(g, res, sl[i], 0.01, 1e-7, 0, orc=orcs[i],
                                            with_r=False)))
                res_r = ctx.result(qr, release=True)
                check_query(g, res_r, sl[i], 0.01, 1e-7, 0, orc=orcs[i])
                check_same(g, res_r, res)
            assert strict_report(name, reps) == 16
            if fixed:
                assert tune["plain_bin_min_edges"] == fixed
                assert sum(x["bin_rounds"] for x in infos) >= 16
        finally:
            ctx.close()


def test_plain_rmat22_learned_bin_launches(plc, g22):
    """With the binning threshold left to the library, a query's first chunk
    queues the binned form's second pass only at the launches where the last
    queries had rounds of that size.  The same 16 queries twice: in the
    second pass every one of them bins exactly the rounds that a context
    with the threshold fixed at the same 524288 edges bins (their own reports
    selected the launches), and both passes give the fixed context's results
    (counters exactly, p and r within the tolerance, the sweep modulo
    near-ties)."""
    g = g22
    sl = [int(s) for s in synth.uniform_seeds(g, 16, seed=2)]
    out = {}
    for fixed in (524288, 0):
        ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20),
                          bin_min_edges=fixed)
        try:
            hg = ctx.load_graph(g.off, g.nbr)
            passes = []
            for rep in range(1 if fixed else 2):
                ids, infos = ctx.run(hg, sl, 0.01, 1e-7)
                passes.append((infos, ctx.results(ids, release=True)))
            out[fixed] = passes
        finally:
            ctx.close()
    (fi, fr), = out[524288]
    say("fixed threshold: binned rounds per query", [x["bin_rounds"] for x in fi])
    assert sum(x["bin_rounds"] for x in fi) >= 16
    for k, (infos, res) in enumerate(out[0]):
        say("learned, pass", k, "binned rounds per query", [x["bin_rounds"] for x in infos])
        for a, b in zip(res, fr):
            check_same(g, a, b)
    assert [x["bin_rounds"] for x in out[0][1][0]] == [x["bin_rounds"] for x in fi]


def test_plain_rmat22_support_above_2_21_with_residual(plc, g22):
    """PR-Nibble from the benchmark's first seed at eps 1e-8: a support of
    about 2.4 M vertices (more block-sort tiles than the launch has
    workgroups, so the residual's gather runs on workgroups that sorted
    tiles, and the deepest merge passes) and about 1.8 M nonzeros of r,
    checked against the oracle with the residual."""
    g = g22
    x = int(synth.uniform_seeds(g, 16, seed=2)[0])
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        say("case plain 2^22 seed", x, "alpha 0.01 eps 1e-8")
        ids, infos = ctx.run(hg, [x], 0.01, 1e-8)
        res = ctx.result(ids[0], release=True)
        say("support", infos[0]["support"], "r nonzeros", infos[0]["r_nnz"])
        assert infos[0]["support"] > 512 * 4096
        assert infos[0]["r_nnz"] > (1 << 20)
        rep = check_query(g, res, x, 0.01, 1e-8, 0)
        say("report", rep)
    finally:
        ctx.close()


def _batched(plc, g, compact):
    qs = synth.batched_queries(g, 256, seed=2, eps_lo=1e-7, eps_hi=1e-5)
    tables = (8 << 30) if compact else 0
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, 256, compact=compact,
                                              table_bytes=tables) + (512 << 20),
                      compact=compact)
    name = "batched 2^22 %s" % ("compact" if compact else "dense")
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 256) == 256
        tune = ctx.autotune(hg, qs.seeds, qs.alpha, qs.eps, plc.PLC_TUNE_BATCH)
        say(name, "shapes", tune["batch_self"], tune["batch_scatter"])
        ids, infos = ctx.run_batched(hg, qs.seeds, qs.alpha, qs.eps)
        sample = set(np.argsort(qs.eps)[::4].tolist())  # every 4th eps, smallest to largest
        reps = []
        for i, qid in enumerate(ids):
            res = ctx.result(qid, release=True)
            check_properties(g, res, float(qs.eps[i]))
            if i in sample:
                reps.append((i, check_query(g, res, int(qs.seeds[i]), float(qs.alpha[i]),
                                            float(qs.eps[i]), 0)))
        assert strict_report(name, reps) == len(sample) == 64
    finally:
        ctx.close()


def test_batched_rmat22_bench_shapes(plc, g22):
    _batched(plc, g22, compact=False)


def test_batched_compact_rmat22_bench_shapes(plc, g22):
    _batched(plc, g22, compact=True)


def test_serving_rmat24_bench_shapes(plc):
    from paper_1604_07515_amd import serve
    g = synth.rmat(24, 16, seed=1)
    say("serving graph 2^24 arcs", g.arcs)
    rng = np.random.default_rng(2)
    nq = 512
    seeds = synth.degree_weighted_seeds(g, 40000, rng)[:nq]
    eps = (10.0 ** rng.uniform(-7, -4, 40000))[:nq]
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, 256, compact=True,
                                              table_bytes=8 << 30) + (1 << 30), compact=True)
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 256) == 256
        ctx.autotune(hg, seeds[:128], 0.01, eps[:128], plc.PLC_TUNE_BATCH)
        arr = serve.poisson_arrivals(nq, 8000.0, np.random.default_rng(3))
        rep = serve.serve(ctx, hg, seeds, 0.01, eps, arr, release=False,
                          flags=plc.PLC_QF_NO_RESIDUAL)
        say("serving 2^24: %.0f q/s, max in flight %d" % (rep.queries_per_s, rep.max_in_flight))
        assert rep.max_in_flight > 1
        results = [ctx.result(int(qid), release=True) for qid in rep.ids]
        for i, res in enumerate(results):
            check_properties(g, res, float(eps[i]), with_r=False)
        reps = []
        for i in range(0, nq, 16):
            say("serving 2^24 oracle query", i)
            reps.append((i, check_query(g, results[i], int(seeds[i]), 0.01, float(eps[i]), 0,
                                        with_r=False)))
        assert strict_report("serving 2^24", reps) == len(reps)
        for i in (0, 101, 255):
            ids1, _ = ctx.run_batched(hg, [int(seeds[i])], 0.01, float(eps[i]),
                                      flags=plc.PLC_QF_NO_RESIDUAL)
            check_same(g, ctx.result(ids1[0], release=True), results[i])
    finally:
        ctx.close()


def test_nibble_support_above_2_21(plc, g22):
    """Nibble (Sec. 3.2) from vertex 0 (the top hub) with T = 2 and eps
    1e-300 (nothing truncated): p_2 covers every vertex within two hops,
    2,208,937 of them, and the sweep over it is checked against the oracle.

    Tolerance: p_1 has one addend per vertex, so both sides form the
    addends of step 2 bit for bit and differ only in the order of the sums:
    p_2[w] adds at most d(w) + 1 positive terms, and two orders of k positive
    terms differ by at most 2 (k - 1) u relative (u = 2^-53), which passes
    1e-12 once k exceeds about 4500.  Each vertex is held to the larger of
    1e-12 and 2 d(w) u; the test reports how many needed more than 1e-12."""
    g = g22
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (512 << 20))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        qid, info = ctx.run_nibble(hg, 0, 1e-300, 2)
        say("nibble 2^22 hub: support", info["support"], "kstar", info["kstar"])
        assert info["support"] > (1 << 21)
        orc = oracle.nibble(g.off, g.nbr, 0, 1e-300, 2)
        res = ctx.result(qid, release=True)
        tol = np.maximum(RTOL, 2.0 * g.deg.astype(np.float64) * 2.0 ** -53)
        p = res.dense_p(g.n)
        sup = orc.p > 0
        err = np.abs(p[sup] - orc.p[sup]) / orc.p[sup]
        say("nibble p: max rel err %.3g, %d of %d vertices above 1e-12 (max degree there %d)" % (
            err.max(), int((err > RTOL).sum()), int(sup.sum()),
            int(g.deg[np.flatnonzero(sup)[err > RTOL]].max(initial=0))))
        rep = check_nibble(g, res, orc, rtol=tol)
        say("nibble report", rep)
    finally:
        ctx.close()
