"""GPU tests of the batched path: many queries per launch, each result equal
to the oracle's and to the same query run alone (through the C ABI)."""
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


@pytest.fixture(scope="module")
def setup(plc):
    g = synth.rmat(14, 8, seed=6)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                      + plc.batch_arena_bytes(g.n, g.arcs, 64))
    hg = ctx.load_graph(g.off, g.nbr, validate=True)
    got = ctx.batch_reserve(hg, 64)
    assert got == 64
    yield g, ctx, hg
    ctx.close()


def mixed_queries(g, k, seed):
    q = synth.batched_queries(g, k, seed=seed, eps_lo=1e-7, eps_hi=1e-4)
    rng = np.random.default_rng(seed + 100)
    rules = rng.integers(0, 2, k)
    return q.seeds, q.alpha, q.eps, rules


def test_batched_mix_matches_oracle(setup):
    """160 queries through 64 slots (continuous admission), mixed eps, alpha and rule."""
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 160, seed=21)
    say("batched mix of", len(seeds))
    ids, infos = ctx.run_batched(hg, seeds, alpha, eps, rules)
    for i, qid in enumerate(ids):
        res = ctx.result(qid, release=True)
        check_query(g, res, int(seeds[i]), float(alpha[i]), float(eps[i]), int(rules[i]))


def test_alone_equals_in_mix(setup):
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 48, seed=33)
    ids_mix, _ = ctx.run_batched(hg, seeds, alpha, eps, rules)
    mix = [ctx.result(i, release=True) for i in ids_mix]
    for j in (0, 7, 19, 47):
        ids1, _ = ctx.run_batched(hg, [seeds[j]], alpha[j], eps[j], rules[j])
        alone = ctx.result(ids1[0], release=True)
        check_same(g, alone, mix[j])


def test_batched_equals_plain(setup):
    g, ctx, hg = setup
    seeds = synth.uniform_seeds(g, 12, seed=44)
    ids_b, infos_b = ctx.run_batched(hg, seeds, 0.01, 1e-6)
    ids_p, infos_p = ctx.run(hg, seeds, 0.01, 1e-6)
    for a, b in zip(ids_b, ids_p):
        check_same(g, ctx.result(a, release=True), ctx.result(b, release=True))


def test_submit_progress_poll(setup, plc):
    g, ctx, hg = setup
    seeds = synth.uniform_seeds(g, 5, seed=55)
    ids = ctx.submit(hg, seeds, 0.02, 1e-5)
    assert all(i > 0 for i in ids)
    assert not ctx.poll(ids[0])
    with pytest.raises(plc.PlcError) as e:
        ctx.result(ids[0])
    assert e.value.code == plc.PLC_E_NOTREADY
    steps = 0
    while ctx.progress(hg) > 0:
        steps += 1
        assert steps < 10000
    assert all(ctx.poll(i) for i in ids)
    for i, s in zip(ids, seeds):
        check_query(g, ctx.result(i, release=True), int(s), 0.02, 1e-5, 0)
    # invalid queries get id 0 and an error, valid ones in the same call still run
    ids = ctx.submit(hg, [int(seeds[0]), -3], 0.02, 1e-5, check=False)
    assert ids[0] > 0 and ids[1] == 0
    while ctx.progress(hg) > 0:
        pass
    ctx.release(ids[0])


def test_batched_rmat16_large_supports(plc):
    """2^16 graph, 32 queries with eps down to 1e-7 (supports up to the whole component)."""
    g = synth.rmat(16, 8, seed=1)
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, 32)) as ctx:
        hg = ctx.load_graph(g.off, g.nbr)
        assert ctx.batch_reserve(hg, 32) == 32
        q = synth.batched_queries(g, 32, seed=5, eps_lo=1e-7, eps_hi=1e-5)
        seeds = np.concatenate([[0], q.seeds[1:]])
        ids, infos = ctx.run_batched(hg, seeds, q.alpha, q.eps)
        for i, qid in enumerate(ids):
            res = ctx.result(qid, release=True)
            check_query(g, res, int(seeds[i]), float(q.alpha[i]), float(q.eps[i]), 0)


def test_reserve_limited_by_arena(plc):
    g = synth.rmat(12, 8, seed=2)
    base = plc.plain_arena_bytes(g.n, g.arcs)
    with plc.Context(arena_bytes=base + plc.batch_arena_bytes(g.n, g.arcs, 4)) as ctx:
        hg = ctx.load_graph(g.off, g.nbr)
        got = ctx.batch_reserve(hg, 1000)
        assert 1 <= got < 1000
        # more queries than slots: admission continues as slots retire
        seeds = synth.uniform_seeds(g, got + 37, seed=3)
        ids, infos = ctx.run_batched(hg, seeds, 0.01, 1e-4)
        assert all(x["status"] == 0 for x in infos)
        for i in ids:
            ctx.release(i)


def test_autotune_keeps_results(setup, plc):
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 24, seed=77)
    tune = ctx.autotune(hg, seeds[:8], alpha[:8], eps[:8],
                        plc.PLC_TUNE_PLAIN | plc.PLC_TUNE_BATCH)
    # plain self x scatter x sweep, three binning thresholds, batched self x scatter
    assert tune["candidates"] == 5 * 4 * 2 + 3 + 2 * 4
    assert tune["plain_bin_min_edges"] in (524288, 4 * 524288, -1)
    for key in ("plain_self", "plain_scatter", "plain_sweep", "batch_self", "batch_scatter"):
        assert tune[key] > 0
    ids, _ = ctx.run_batched(hg, seeds, alpha, eps, rules)
    for i, qid in enumerate(ids):
        check_query(g, ctx.result(qid, release=True), int(seeds[i]), float(alpha[i]),
                    float(eps[i]), int(rules[i]))
    ids, _ = ctx.run(hg, seeds[:6], alpha[:6], eps[:6], rules[:6])
    for i, qid in enumerate(ids):
        check_query(g, ctx.result(qid, release=True), int(seeds[i]), float(alpha[i]),
                    float(eps[i]), int(rules[i]))


def test_wait_and_bytes_estimate(setup, plc):
    """plc_wait drives the engine until one query is done; the byte estimate
    bounds each query's slot state plus result block."""
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 12, seed=55)
    ids = ctx.submit(hg, seeds, alpha, eps, rules)
    assert not ctx.wait(ids[11], 0)          # nothing stepped yet: times out at once
    assert ctx.wait(ids[11])
    assert ctx.poll(ids[11])
    slot = 40 * g.n
    for i, qid in enumerate(ids):
        assert ctx.wait(qid, 60_000_000)
        res = ctx.result(qid, release=True)
        check_query(g, res, int(seeds[i]), float(alpha[i]), float(eps[i]), int(rules[i]))
        est = ctx.query_bytes_estimate(hg, int(seeds[i]), float(alpha[i]), float(eps[i]),
                                       int(rules[i]))
        assert est >= slot + 12 * (res.info["support"] + res.info["r_nnz"])
    assert ctx.query_bytes_estimate(hg, -1, 0.01, 1e-4) == 0
    with pytest.raises(plc.PlcError):
        ctx.wait(ids[0])                       # released: unknown id


@pytest.mark.parametrize("graphs", [True, False])
def test_batched_launch_modes(plc, graphs):
    """The batched round as a replayed graph and as direct launches."""
    g = synth.rmat(12, 8, seed=12)
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.batch_arena_bytes(g.n, g.arcs, 16), graphs=graphs) as c:
        hg = c.load_graph(g.off, g.nbr)
        assert c.batch_reserve(hg, 16) == 16
        seeds, alpha, eps, rules = mixed_queries(g, 40, seed=77)
        say("case batched launch mode graphs=%s" % graphs)
        c.timing(True)
        ids, infos = c.run_batched(hg, seeds, alpha, eps, rules)
        tm = c.timing_get()
        c.timing(False)
        assert tm["scatter"]["launches"] > 0 and tm["scatter"]["ms"] > 0
        assert tm["scatter"]["units"] == sum(i["edges"] for i in infos)
        for i, qid in enumerate(ids):
            check_query(g, c.result(qid, release=True), int(seeds[i]), float(alpha[i]),
                        float(eps[i]), int(rules[i]))


def test_batched_flags_and_device_time(setup, plc):
    """The batched path honours PLC_QF_NO_RESIDUAL and reports each query's
    device time from admission to its sweep's argmin."""
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 24, seed=41)
    ids_a, infos_a = ctx.run_batched(hg, seeds, alpha, eps, rules)
    ids_b, infos_b = ctx.run_batched(hg, seeds, alpha, eps, rules, flags=plc.PLC_QF_NO_RESIDUAL)
    for i, (qa, qb) in enumerate(zip(ids_a, ids_b)):
        ia, ib = infos_a[i], infos_b[i]
        a = ctx.result(qa, release=True)
        b = ctx.result(qb, release=True)
        assert ib["flags"] == plc.PLC_QF_NO_RESIDUAL and ib["r_nnz"] == ia["r_nnz"]
        assert len(b.r_ids) == 0
        check_same(g, a, b)
        assert 0 < ia["device_ns"] < 10 ** 10 and 0 < ib["device_ns"] < 10 ** 10


def test_result_copy_many_matches_one_by_one(setup, plc):
    """plc_result_copy_many returns, for several results at once, what
    plc_result_copy returns for each (with and without the residual, and
    across a staging-memory growth); unknown ids are refused."""
    g, ctx, hg = setup
    seeds, alpha, eps, rules = mixed_queries(g, 40, seed=91)
    for flags in (0, plc.PLC_QF_NO_RESIDUAL):
        ids, _ = ctx.run_batched(hg, seeds, alpha, eps, rules, flags=flags)
        many = ctx.results(ids)
        for i, (qid, m) in enumerate(zip(ids, many)):
            one = ctx.result(qid, release=True)
            assert m.info == one.info
            for a, b in ((m.sweep_ids, one.sweep_ids), (m.sweep_p, one.sweep_p),
                         (m.r_ids, one.r_ids), (m.r_vals, one.r_vals)):
                np.testing.assert_array_equal(a, b)
            check_query(g, m, int(seeds[i]), float(alpha[i]), float(eps[i]), int(rules[i]),
                        with_r=flags == 0)
    with pytest.raises(plc.PlcError):
        ctx.results([123456789])
