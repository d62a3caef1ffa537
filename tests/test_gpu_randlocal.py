"""The paper's randLocal input at full size (n = 10^7, five drawn neighbours
per vertex, offsets favouring near ids, 49.1 M distinct edges), alpha 0.01,
eps 1e-7, optimized rule -- the setting of the paper's PR-Nibble timings.
The plain path against the oracle on two seeds: hundreds of mostly small
rounds, so the rounds run inside the self launch as well as the scatter."""
import sys

import pytest

import synth
from parity import check_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    g = synth.rand_local(10_000_000)
    say("randlocal: n", g.n, "arcs", g.arcs)
    return g


def test_randlocal_full(g):
    import paper_1604_07515_amd as plc
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20)) as c:
        hg = c.load_graph(g.off, g.nbr)
        for seed in (0, 4_000_321):
            say("case randlocal seed", seed)
            ids, infos = c.run(hg, [seed], 0.01, 1e-7)
            out = check_query(g, c.result(ids[0], release=True), seed, 0.01, 1e-7, 0)
            say("  rounds", out["rounds"], "support", out["support"], "ties", out["tie_push"],
                out["tie_sweep"], "loop rounds", infos[0]["loop_rounds"])


def test_randlocal_batched_compact(g):
    """Eight queries at once through the compact-table engine (the dense
    per-query state would not fit 10^7 vertices per slot on one GPU at any
    useful slot count), each against the oracle."""
    import paper_1604_07515_amd as plc
    seeds = [int(x) for x in synth.uniform_seeds(g, 8, seed=5)]
    slots = 8
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=True,
                                             table_bytes=4 << 30), compact=True) as c:
        hg = c.load_graph(g.off, g.nbr)
        assert c.batch_reserve(hg, slots) == slots
        say("case randlocal batched seeds", seeds)
        ids, infos = c.run_batched(hg, seeds, 0.01, 1e-7)
        for i, qid in enumerate(ids):
            out = check_query(g, c.result(qid, release=True), seeds[i], 0.01, 1e-7, 0)
            say("  seed", seeds[i], "rounds", out["rounds"], "support", out["support"])
