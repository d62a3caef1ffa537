"""Parity on the large skewed graph: R-MAT 2^26 (ef 16, ~2.1 G arcs, max
degree ~1 M), seeds including the top-degree hubs, eps log-uniform in
[1e-8, 1e-6], alpha 0.01, through the compact-table engine (dense slots would
cost 2.7 GB each at this size).

48 queries (40 uniform seeds + the 8 highest-degree hubs) run in one batch;
every result is checked for the properties that hold at any size (mass,
termination, sweep order, the reported cut and volume recounted from the
cluster), and a sample -- including a hub and the heaviest eps -- against the
oracle.  The benchmark's 1024-seed run on this graph is `bench.py --only large`.
On the same graph, a Nibble query from the top hub sweeps a support of more
than 10^7 vertices against the oracle.
"""
import sys

import numpy as np
import pytest

import synth
import oracle
from parity import RTOL, check_nibble, check_properties, check_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g26():
    g = synth.rmat(26, 16, seed=1)
    say("graph 2^26 arcs", g.arcs, "maxdeg", int(g.deg.max()))
    return g


def test_large_rmat26_sampled(g26):
    import paper_1604_07515_amd as plc
    g = g26
    hubs = np.argsort(-g.deg, kind="stable")[:8]
    seeds = np.concatenate([synth.uniform_seeds(g, 40, seed=12), hubs])
    eps = 10.0 ** np.random.default_rng(12).uniform(-8, -6, len(seeds))
    eps[40] = 1e-6  # the top hub, at the largest eps
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, 64, compact=True,
                                             table_bytes=80 << 30), compact=True) as c:
        hg = c.load_graph(g.off, g.nbr)
        assert c.batch_reserve(hg, 64) == 64
        say("running", len(seeds), "queries")
        ids, infos = c.run_batched(hg, seeds, 0.01, eps)
        say("edges pushed", sum(i["edges"] for i in infos),
            "max support", max(i["support"] for i in infos))
        # oracle samples: the two largest eps, the top hub, and the heaviest
        # query (by pushed edges) that the oracle finishes in a few seconds
        edges = np.array([i["edges"] for i in infos])
        light = np.flatnonzero(edges[:40] <= 2e8)
        sample = set(np.argsort(-eps[:40])[:2].tolist()) | {40}
        if len(light):
            sample.add(int(light[np.argmax(edges[light])]))
        for i, qid in enumerate(ids):
            res = c.result(qid, release=True)
            check_properties(g, res, float(eps[i]))
            if i in sample:
                say("oracle check of query", i, "seed", int(seeds[i]), "eps", float(eps[i]))
                check_query(g, res, int(seeds[i]), 0.01, float(eps[i]), 0)


def test_nibble_support_above_1e7(g26):
    """A sweep at the C5 scale: Nibble (Sec. 3.2) from the top hub of R-MAT
    2^26 with T = 2 and eps 1e-300 (nothing truncated) covers every vertex
    within two hops of the hub, more than 10^7 of them, and the support's
    sort, volume and cut scans and argmin are checked against the oracle.
    Per-vertex tolerance max(1e-12, 2 d(w) u) as for the 2^22 case: p_2[w]
    sums at most d(w) + 1 addends that both sides form bit for bit."""
    import paper_1604_07515_amd as plc
    g = g26
    x = int(np.argmax(g.deg))
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (1 << 30)) as c:
        hg = c.load_graph(g.off, g.nbr)
        qid, info = c.run_nibble(hg, x, 1e-300, 2)
        say("nibble 2^26 hub %d: support %d, kstar %d, edges %d" % (
            x, info["support"], info["kstar"], info["edges"]))
        assert info["support"] > 10 ** 7
        res = c.result(qid, release=True)
    orc = oracle.nibble(g.off, g.nbr, x, 1e-300, 2)
    say("oracle done")
    tol = np.maximum(RTOL, 2.0 * g.deg.astype(np.float64) * 2.0 ** -53)
    rep = check_nibble(g, res, orc, rtol=tol)
    say("nibble 2^26 report", rep)
