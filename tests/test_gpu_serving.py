"""GPU tests of the serving loop: queries arriving while others run join the
batch at round boundaries, and every result is the same as the query alone
(and as the oracle)."""
import sys

import numpy as np
import pytest

import synth
from parity import check_query, check_same

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def plc():
    import paper_1604_07515_amd as plc
    return plc


def test_poisson_arrivals_join_running_batch(plc):
    from paper_1604_07515_amd import serve
    g = synth.rmat(13, 8, seed=8)
    rng = np.random.default_rng(9)
    k = 60
    seeds = synth.degree_weighted_seeds(g, k, rng)
    eps = 10.0 ** rng.uniform(-7, -4, k)
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, 8)) as ctx:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 8) == 8
        # arrivals spread over a few ms so that some land while others run
        arr = serve.poisson_arrivals(k, 20000.0, rng)
        rep = serve.serve(ctx, hg, seeds, 0.01, eps, arr, release=False)
        say("serve: steps", rep.steps, "max in flight", rep.max_in_flight,
            "p50 ms", rep.percentile_ms(50))
        assert np.all(np.isfinite(rep.latency_s)) and np.all(rep.latency_s >= 0)
        assert rep.max_in_flight > 8  # more queries than slots were in the system at once
        mixed = [ctx.result(int(i), release=True) for i in rep.ids]
        for i in range(k):
            check_query(g, mixed[i], int(seeds[i]), 0.01, float(eps[i]), 0)
        for i in (0, 13, 31, 59):
            ids, _ = ctx.run_batched(hg, [seeds[i]], 0.01, eps[i])
            check_same(g, ctx.result(ids[0], release=True), mixed[i])


def test_saturation_closed_loop(plc):
    from paper_1604_07515_amd import serve
    g = synth.rmat(12, 8, seed=10)
    rng = np.random.default_rng(11)
    seeds = synth.degree_weighted_seeds(g, 100, rng)
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, 16)) as ctx:
        hg = ctx.load_graph(g.off, g.nbr)
        ctx.batch_reserve(hg, 16)
        rep = serve.saturation(ctx, hg, seeds, 0.01, 1e-5)
        assert rep.queries_per_s > 0 and np.all(np.isfinite(rep.latency_s))
