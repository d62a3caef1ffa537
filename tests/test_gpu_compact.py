"""GPU tests of the batch engine's compact layout (per-query open-addressing
tables taken from the arena and grown between rounds), through the C ABI:
results equal to the oracle's and to the dense layout's, tables that grow
from their smallest size, admission and growth under a tight arena, and a
query that cannot fit failing alone."""
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


def mixed_queries(g, k, seed, eps_lo=1e-7, eps_hi=1e-4):
    q = synth.batched_queries(g, k, seed=seed, eps_lo=eps_lo, eps_hi=eps_hi)
    rules = np.random.default_rng(seed + 100).integers(0, 2, k)
    return q.seeds, q.alpha, q.eps, rules


def context(plc, g, slots, compact, table_bytes=256 << 20, graphs=True):
    c = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                    + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=compact,
                                            table_bytes=table_bytes if compact else 0),
                    compact=compact, graphs=graphs)
    hg = c.load_graph(g.off, g.nbr)
    assert c.batch_reserve(hg, slots) == slots
    return c, hg


@pytest.mark.parametrize("graphs", [True, False])
def test_compact_mix_matches_oracle(plc, graphs):
    g = synth.rmat(14, 8, seed=6)
    c, hg = context(plc, g, 64, True, graphs=graphs)
    with c:
        seeds, alpha, eps, rules = mixed_queries(g, 160, seed=21)
        say("compact mix graphs=%s" % graphs)
        ids, infos = c.run_batched(hg, seeds, alpha, eps, rules)
        for i, qid in enumerate(ids):
            check_query(g, c.result(qid, release=True), int(seeds[i]), float(alpha[i]),
                        float(eps[i]), int(rules[i]))


def test_compact_equals_dense(plc):
    g = synth.rmat(15, 8, seed=2)
    seeds, alpha, eps, rules = mixed_queries(g, 96, seed=5)
    out = {}
    for compact in (False, True):
        c, hg = context(plc, g, 32, compact)
        with c:
            say("layout compact=%s" % compact)
            ids, _ = c.run_batched(hg, seeds, alpha, eps, rules)
            out[compact] = [c.result(i, release=True) for i in ids]
    for a, b in zip(out[False], out[True]):
        check_same(g, a, b)


def test_compact_tables_grow_from_smallest(plc):
    """Degree-1 seeds start with the smallest table (256 records) and, at eps
    1e-7 on 2^16 vertices, touch most of their component: many growths."""
    g = synth.rmat(16, 8, seed=1)
    seeds = np.flatnonzero(g.deg == 1)[:12]
    c, hg = context(plc, g, 16, True)
    with c:
        say("compact growth seeds", seeds.tolist())
        ids, infos = c.run_batched(hg, seeds, 0.01, 1e-7)
        for i, qid in enumerate(ids):
            res = c.result(qid, release=True)
            assert res.info["r_nnz"] + res.info["support"] > 256
            check_query(g, res, int(seeds[i]), 0.01, 1e-7, 0)


def tight_context(plc, g, slots, table_mib):
    """A compact context whose arena leaves about `table_mib` MiB for tables
    beyond the result headroom (64 MiB)."""
    probe = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                        + plc.batch_arena_bytes(g.n, g.arcs, slots, compact=True),
                        compact=True)
    hg = probe.load_graph(g.off, g.nbr)
    probe.batch_reserve(hg, slots)
    total, _ = probe.arena_free()
    used = probe.arena_bytes - total
    probe.close()
    c = plc.Context(arena_bytes=used + (64 << 20) + (table_mib << 20), compact=True)
    hg = c.load_graph(g.off, g.nbr)
    assert c.batch_reserve(hg, slots) == slots
    return c, hg


def test_compact_tight_arena_holds_and_succeeds(plc):
    """With room for only a few large tables at once, queries wait for memory
    (admission and growth) but every one finishes with the oracle's result."""
    g = synth.rmat(17, 8, seed=3)
    c, hg = tight_context(plc, g, 32, 24)
    with c:
        seeds = synth.uniform_seeds(g, 40, seed=4)
        say("tight arena")
        ids, infos = c.run_batched(hg, seeds, 0.01, 1e-6)
        for i, qid in enumerate(ids):
            assert infos[i]["status"] == 0
            check_query(g, c.result(qid, release=True), int(seeds[i]), 0.01, 1e-6, 0)


def test_compact_query_too_large_fails_alone(plc):
    """A query whose table cannot grow within the arena fails with
    PLC_E_NOMEM once nothing else can free memory; a small query of the same
    batch is unaffected."""
    g = synth.rmat(20, 8, seed=5)
    c, hg = tight_context(plc, g, 4, 8)
    with c:
        small = int(np.flatnonzero(g.deg == 3)[0])
        big = int(np.argmax(g.deg))
        say("too large: small", small, "big", big)
        ids, infos = c.run_batched(hg, [small, big], [0.05, 0.01], [1e-3, 1e-8], check=False)
        assert infos[0]["status"] == 0
        check_query(g, c.result(ids[0], release=True), small, 0.05, 1e-3, 0)
        assert infos[1]["status"] == plc.PLC_E_NOMEM
        c.release(ids[1])
        # the engine stays usable: the small query again
        ids2, infos2 = c.run_batched(hg, [small], 0.05, 1e-3)
        check_query(g, c.result(ids2[0], release=True), small, 0.05, 1e-3, 0)


def test_compact_serving_alone_equals_mix(plc):
    from paper_1604_07515_amd import serve
    g = synth.rmat(13, 8, seed=8)
    c, hg = context(plc, g, 16, True)
    with c:
        rng = np.random.default_rng(9)
        seeds = synth.degree_weighted_seeds(g, 48, rng)
        eps = 10.0 ** rng.uniform(-7, -4, 48)
        arr = serve.poisson_arrivals(48, 3000.0, np.random.default_rng(1))
        rep = serve.serve(c, hg, seeds, 0.01, eps, arr, release=False)
        assert rep.max_in_flight > 1
        mix = [c.result(int(q), release=True) for q in rep.ids]
        for i in range(48):
            check_query(g, mix[i], int(seeds[i]), 0.01, float(eps[i]), 0)
        for i in (0, 17, 47):
            ids1, _ = c.run_batched(hg, [int(seeds[i])], 0.01, float(eps[i]))
            check_same(g, c.result(ids1[0], release=True), mix[i])


def test_compact_first_table_does_not_fit(plc):
    """Less room beyond the result headroom than the query's first table: it
    cannot be admitted and, with nothing else running, fails at once with
    PLC_E_NOMEM."""
    g = synth.rmat(20, 8, seed=5)
    # the hub's first table: 4/3 (d + 1) = 52948 records rounded up to 53248,
    # 36 B each (1.83 MiB)
    c, hg = tight_context(plc, g, 4, 1)
    with c:
        seed = int(np.argmax(g.deg))
        ids, infos = c.run_batched(hg, [seed], 0.01, 1e-4, check=False)
        assert infos[0]["status"] == plc.PLC_E_NOMEM
        c.release(ids[0])
