"""GPU parity of the plain path (one query at a time) against the oracle.

Every call goes through the C ABI of libplc (via the ctypes binding).
Inputs are seeded synthetic graphs; sizes span several scan blocks, edge
tiles and radix tiles with ragged tails.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_query, check_same

pytestmark = pytest.mark.gpu

OPT, ORIG = 0, 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def plc():
    import paper_1604_07515_amd as plc
    return plc


@pytest.fixture(scope="module")
def ctx(plc):
    c = plc.Context(arena_bytes=3 << 30)
    yield c
    c.close()


GRAPHS = {
    "rmat10": lambda: synth.rmat(10, 8, seed=3),
    "rmat13": lambda: synth.rmat(13, 8, seed=4),
    "rmat16": lambda: synth.rmat(16, 8, seed=1),
    "barbell12": lambda: synth.barbell(12),
    "star300": lambda: synth.star(300),
    "k40": lambda: synth.complete(40),
    "torus12": lambda: synth.torus3d(12),
    "k2": lambda: synth.path(2),
}
_cache = {}


def graph(ctx, name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, ctx.load_graph(g.off, g.nbr, validate=True))
    return _cache[name]


CASES = []
for gname in ("rmat10", "rmat13", "barbell12", "star300", "k40", "torus12", "k2"):
    for rule in (OPT, ORIG):
        for eps in (1e-3, 1e-5, 1e-7):
            CASES.append((gname, rule, eps))


@pytest.mark.parametrize("gname,rule,eps", CASES)
def test_parity_small(ctx, gname, rule, eps):
    g, hg = graph(ctx, gname)
    seeds = [int(s) for s in synth.uniform_seeds(g, 2, seed=7)]
    alpha = 0.01 if rule == OPT else 0.05
    say("case", gname, rule, eps, seeds)
    ids, infos = ctx.run(hg, seeds, alpha, eps, rule)
    for qid, s in zip(ids, seeds):
        res = ctx.result(qid, release=True)
        check_query(g, res, s, alpha, eps, rule)


def test_parity_rmat16_seed0_full(ctx):
    """2^16 vertices, avg degree ~16, alpha=0.01, eps=1e-7, seed 0 (largest component)."""
    g, hg = graph(ctx, "rmat16")
    x = synth.largest_component_min_vertex(g)
    say("case rmat16 seed", x)
    ids, infos = ctx.run(hg, [x], 0.01, 1e-7, OPT)
    res = ctx.result(ids[0], release=True)
    rep = check_query(g, res, x, 0.01, 1e-7, OPT)
    say("report", rep)
    assert rep["rounds"] > 50 and rep["support"] > 30000


def test_same_query_twice_is_identical_and_state_resets(ctx):
    g, hg = graph(ctx, "rmat13")
    seeds = [int(s) for s in synth.uniform_seeds(g, 3, seed=11)]
    say("case repeat", seeds)
    ids1, _ = ctx.run(hg, seeds, 0.02, 1e-6, OPT)
    ids2, _ = ctx.run(hg, seeds[::-1], 0.02, 1e-6, OPT)
    r1 = [ctx.result(i, release=True) for i in ids1]
    r2 = [ctx.result(i, release=True) for i in ids2][::-1]
    for a, b, s in zip(r1, r2, seeds):
        check_same(g, a, b)
        check_query(g, b, s, 0.02, 1e-6, OPT)


def test_invalid_queries_rejected(ctx, plc):
    g = synth.from_edges(6, [(0, 1), (1, 2), (2, 3)])  # 4 and 5 isolated
    hg = ctx.load_graph(g.off, g.nbr, validate=True)
    bad = [(4, 0.01, 1e-4), (9, 0.01, 1e-4), (-1, 0.01, 1e-4), (0, 0.0, 1e-4), (0, 1.0, 1e-4),
           (0, 0.01, 0.0), (0, 0.01, float("nan")), (0, 0.01, float("inf"))]
    for s, a, e in bad:
        ids, infos = ctx.run(hg, [s], a, e, OPT, check=False)
        assert ids[0] == 0 and infos[0]["status"] == plc.PLC_E_INVALID
    # a good query in the same call still runs
    ids, infos = ctx.run(hg, [4, 0], [0.01, 0.01], [1e-4, 1e-4], OPT, check=False)
    assert infos[0]["status"] == plc.PLC_E_INVALID and infos[1]["status"] == 0
    res = ctx.result(ids[1], release=True)
    check_query(g, res, 0, 0.01, 1e-4, OPT)
    hg.free()


def test_invalid_graphs_rejected(ctx, plc):
    g = synth.path(5)
    nbr = g.nbr.copy()
    nbr[0] = 0  # self-loop
    with pytest.raises(plc.PlcError) as e:
        ctx.load_graph(g.off, nbr, validate=True)
    assert e.value.code == plc.PLC_E_INVALID
    off = g.off.copy()
    off[2] = off[3] + 1  # not monotone
    with pytest.raises(plc.PlcError):
        ctx.load_graph(off, g.nbr)


def test_watchdog_limit(plc):
    g = synth.path(2)
    with plc.Context(arena_bytes=64 << 20, max_rounds=5) as c:
        hg = c.load_graph(g.off, g.nbr)
        ids, infos = c.run(hg, [0], 0.01, 1e-7, OPT, check=False)
        assert infos[0]["status"] == plc.PLC_E_LIMIT and infos[0]["rounds"] == 5
        res = c.result(ids[0], release=True)
        part = oracle.prnibble(g.off, g.nbr, 0, 0.01, 1e-7, OPT, max_rounds=5)
        assert np.allclose(res.dense_p(2), part.p, rtol=1e-12, atol=0)


def test_arena_exhausted(plc):
    g = synth.rmat(15, 8, seed=1)  # needs several MiB of plain-path state
    with plc.Context(arena_bytes=1 << 20) as c:
        with pytest.raises(plc.PlcError) as e:
            c.load_graph(g.off, g.nbr)
        assert e.value.code == plc.PLC_E_NOMEM


def test_seed_above_threshold_pushes_once(ctx):
    g, hg = graph(ctx, "star300")
    ids, infos = ctx.run(hg, [0], 0.01, 0.5, OPT)  # eps * d(0) = 150 > 1
    res = ctx.result(ids[0], release=True)
    assert infos[0]["rounds"] == 1 and infos[0]["pushes"] == 1
    check_query(g, res, 0, 0.01, 0.5, OPT)


@pytest.mark.parametrize("graphs", [True, False])
def test_launch_modes_agree_and_time(plc, graphs):
    """Replayed HIP graphs and direct launches run the same kernels: equal
    results (modulo the order of atomic additions), and the per-kernel timing
    counts the launches that did work in both modes: one self launch per
    working step, one scatter launch per round not run inside a self launch
    (small rounds run there, by one workgroup)."""
    g = synth.rmat(13, 8, seed=4)
    seeds = [int(s) for s in synth.uniform_seeds(g, 6, seed=19)]
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (64 << 20),
                     graphs=graphs) as c:
        hg = c.load_graph(g.off, g.nbr)
        say("case launch mode graphs=%s" % graphs, seeds)
        c.timing(True)
        ids, infos = c.run(hg, seeds, 0.01, 1e-6)
        tm = c.timing_get()
        c.timing(False)
        rounds = sum(i["rounds"] for i in infos)
        looped = sum(i["loop_rounds"] for i in infos)
        assert 0 < looped < rounds
        assert tm["scatter"]["launches"] == rounds - looped
        assert tm["self"]["launches"] == sum(i["launches"] for i in infos)
        assert tm["scatter"]["units"] == sum(i["edges"] - i["loop_edges"] for i in infos)
        for i in infos:
            # each working self launch either runs rounds itself or builds
            # one round's entries for the scatter launch, or both
            assert i["rounds"] - i["loop_rounds"] <= i["launches"] <= i["rounds"]
        assert tm["scatter"]["ms"] > 0 and tm["sweep"]["launches"] == len(seeds)
        for qid, s in zip(ids, seeds):
            check_query(g, c.result(qid, release=True), s, 0.01, 1e-6, OPT)
        # a second pass re-uses the recorded graphs (timing off: other graphs)
        ids2, infos2 = c.run(hg, seeds, 0.01, 1e-6)
        for qid, s in zip(ids2, seeds):
            check_query(g, c.result(qid, release=True), s, 0.01, 1e-6, OPT)


def test_int32_offsets_rmat16_seed0(plc):
    """R-MAT 2^16 with int32 CSR offsets (the 32-bit load path): seed 0 of the
    largest component, alpha 0.01, eps 1e-7, against the oracle; the same
    result as the 64-bit load."""
    g = synth.rmat(16, 8, seed=1)
    x = synth.largest_component_min_vertex(g)
    out = []
    for off in (g.off.astype(np.int32), g.off.astype(np.int64)):
        with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (64 << 20)) as c:
            hg = c.load_graph(off, g.nbr, validate=True)
            ids, _ = c.run(hg, [x], 0.01, 1e-7)
            out.append(c.result(ids[0], release=True))
    check_query(g, out[0], x, 0.01, 1e-7, OPT)
    check_same(g, out[0], out[1])


def test_sweep_queued_behind_push(plc):
    """The sweep is queued after each push chunk for the largest recent
    support and runs only if the push ended within that bound.  In a fresh
    context: tiny queries (bound 1024), a query whose support exceeds it (the
    queued sweep stands aside, an exact one follows), a tiny query under the
    grown bound, and a 745-round push on a path (several chunks, the sweeps
    queued behind the unfinished ones stand aside): all match the oracle."""
    g = synth.rmat(13, 8, seed=4)
    pg = synth.path(5000)
    hub = int(np.argmax(g.deg))
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs)
                     + plc.plain_arena_bytes(pg.n, pg.arcs) + (64 << 20)) as c:
        hg = c.load_graph(g.off, g.nbr)
        hp = c.load_graph(pg.off, pg.nbr)
        for eps in (1e-2, 1e-2, 1e-2, 1e-7, 1e-2):
            say("case sweep behind push: rmat13 seed", hub, "eps", eps)
            ids, infos = c.run(hg, [hub], 0.01, eps)
            assert infos[0]["host_ns"] > 0
            if eps == 1e-7:
                assert infos[0]["support"] > 1024
            check_query(g, c.result(ids[0], release=True), hub, 0.01, eps, OPT)
        say("case sweep behind push: path5000 seed 0 eps 1e-8")
        ids, infos = c.run(hp, [0], 0.01, 1e-8)
        assert infos[0]["rounds"] == 745 and infos[0]["launches"] >= 3
        check_query(pg, c.result(ids[0], release=True), 0, 0.01, 1e-8, OPT)


def test_queries_pipelined_in_one_call(plc):
    """In one plc_run call the next query's initialisation and first chunk
    are queued behind the running query's read-back.  When that query still
    needs work (more rounds, or the sweep for a larger support), the queued
    initialisation stands aside and its rounds continue the running query.
    A fresh context and a mix of tiny and large queries (hub with eps 1e-2 /
    1e-7, an invalid seed in between, both rules) cover both cases; every
    result matches the oracle and equals the same query run alone."""
    g = synth.rmat(13, 8, seed=4)
    hub = int(np.argmax(g.deg))
    xs = [int(v) for v in synth.uniform_seeds(g, 4, seed=31)]
    seeds = [hub, xs[0], hub, xs[1], -1, hub, xs[2], hub, xs[3], xs[0]]
    eps = [1e-2, 1e-6, 1e-7, 1e-2, 1e-5, 1e-2, 1e-7, 1e-6, 1e-2, 1e-8]
    rules = [OPT, OPT, OPT, ORIG, OPT, OPT, OPT, ORIG, OPT, OPT]
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (64 << 20)) as c:
        hg = c.load_graph(g.off, g.nbr)
        say("case pipelined plc_run:", list(zip(seeds, eps, rules)))
        ids, infos = c.run(hg, seeds, 0.01, eps, rules, check=False)
        alone = []
        for x, e, r in zip(seeds, eps, rules):
            if x < 0:
                alone.append(None)
                continue
            i1, _ = c.run(hg, [x], 0.01, e, r)
            alone.append(c.result(i1[0], release=True))
        for qid, info, x, e, r, ref in zip(ids, infos, seeds, eps, rules, alone):
            if x < 0:
                assert qid == 0 and info["status"] == plc.PLC_E_INVALID
                continue
            res = c.result(qid, release=True)
            out = check_query(g, res, x, 0.01, e, r)
            if not out["tie_push"]:
                check_same(g, res, ref)
        # both branches of the queued start were taken
        pipes = [info["pipelined"] for info, x in zip(infos, seeds) if x >= 0]
        say("pipelined per query:", pipes)
        assert pipes.count(1) >= 1 and pipes.count(2) >= 1


def test_result_block_does_not_fit(plc):
    """No room for a query's result block: the query reports PLC_E_NOMEM
    with its counters (the sweep itself writes into the library's buffers),
    and the dense state is still reset (a following query, whose neighbours
    the first one touched, matches the oracle)."""
    g = synth.rmat(14, 8, seed=2)
    probe = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs))
    probe.load_graph(g.off, g.nbr)
    total, _ = probe.arena_free()
    used = probe.arena_bytes - total
    probe.close()
    with plc.Context(arena_bytes=used + (16 << 10)) as c:
        hg = c.load_graph(g.off, g.nbr)
        big = int(np.argmax(g.deg))
        say("case result block does not fit: seed", big)
        ids, infos = c.run(hg, [big], 0.01, 1e-7, OPT, check=False)
        assert infos[0]["status"] == plc.PLC_E_NOMEM
        ref = oracle.prnibble(g.off, g.nbr, big, 0.01, 1e-7, OPT)
        assert infos[0]["support"] > 1000
        if ref.min_rel_gap >= 1e-10:
            assert infos[0]["rounds"] == ref.rounds and infos[0]["edges"] == ref.edges
        c.release(ids[0])
        # support 1, touched d + 1: its block fits in the headroom
        small = int(np.flatnonzero(g.deg == 3)[0])
        for _ in range(2):
            ids2, _ = c.run(hg, [small], 0.05, 0.5, OPT)
            check_query(g, c.result(ids2[0], release=True), small, 0.05, 0.5, OPT)


@pytest.mark.parametrize("rule", [OPT, ORIG])
@pytest.mark.parametrize("kind", ["pair", "seven_with_repeats", "wide"])
def test_seed_sets(ctx, plc, rule, kind):
    """plc_run_set against the oracle's seed-set PR-Nibble (unit mass split
    equally over the distinct seeds); the wide set spans several init and
    frontier-scan blocks."""
    g, hg = graph(ctx, "rmat13")
    rng = np.random.default_rng({"pair": 1, "seven_with_repeats": 2, "wide": 3}[kind])
    cand = np.flatnonzero(g.deg > 0)
    k = {"pair": 2, "seven_with_repeats": 7, "wide": 1500}[kind]
    seeds = rng.choice(cand, k, replace=False).astype(np.int32)
    if kind == "seven_with_repeats":
        seeds = np.concatenate([seeds, seeds[:3]])
    eps = 1e-6 if kind != "wide" else 1e-5
    say("case seed set", kind, "rule", rule, "size", len(seeds))
    qid, info = ctx.run_set(hg, seeds, 0.01, eps, rule)
    orc = oracle.prnibble(g.off, g.nbr, seeds, 0.01, eps, rule)
    check_query(g, ctx.result(qid, release=True), int(seeds[0]), 0.01, eps, rule, orc=orc)


def test_seed_set_of_one_is_a_plain_query(ctx, plc):
    g, hg = graph(ctx, "rmat13")
    x = int(np.flatnonzero(g.deg > 2)[7])
    qid, _ = ctx.run_set(hg, [x, x], 0.01, 1e-6)
    ids, _ = ctx.run(hg, [x], 0.01, 1e-6)
    check_same(g, ctx.result(qid, release=True), ctx.result(ids[0], release=True))


def test_seed_set_rejects_bad_input(ctx, plc):
    g, hg = graph(ctx, "rmat13")
    for bad in ([], [g.n], [0, -1]):
        with pytest.raises(plc.PlcError) as e:
            ctx.run_set(hg, np.asarray(bad, dtype=np.int32), 0.01, 1e-6)
        assert e.value.code == plc.PLC_E_INVALID
    iso = np.flatnonzero(g.deg == 0)
    if len(iso):
        with pytest.raises(plc.PlcError):
            ctx.run_set(hg, [int(iso[0])], 0.01, 1e-6)


def test_query_flags_and_device_time(ctx, plc):
    """PLC_QF_NO_RESIDUAL keeps the cluster and p but no residual vector
    (its count is still reported); every result carries the query's device
    time from the kernels' own clock; unknown flags are rejected."""
    g, hg = graph(ctx, "rmat13")
    seeds = [int(s) for s in synth.uniform_seeds(g, 3, seed=17)]
    ids_a, infos_a = ctx.run(hg, seeds, 0.01, 1e-6, OPT)
    ids_b, infos_b = ctx.run(hg, seeds, 0.01, 1e-6, OPT, flags=plc.PLC_QF_NO_RESIDUAL)
    for qa, qb, ia, ib, s in zip(ids_a, ids_b, infos_a, infos_b, seeds):
        a = ctx.result(qa, release=True)
        b = ctx.result(qb, release=True)
        say("flags", ib["flags"], "r_nnz", ib["r_nnz"], "device_ns", ia["device_ns"], ib["device_ns"],
            "host_ns", ia["host_ns"])
        assert ia["flags"] == 0 and ib["flags"] == plc.PLC_QF_NO_RESIDUAL
        assert ib["r_nnz"] == ia["r_nnz"] > 0 and len(b.r_ids) == 0 and len(b.r_vals) == 0
        check_same(g, a, b)
        check_query(g, a, s, 0.01, 1e-6, OPT)
        for info in (ia, ib):
            assert 0 < info["device_ns"] < 10 ** 10
    ids, infos = ctx.run(hg, [seeds[0]], 0.01, 1e-6, OPT, check=False, flags=2)
    assert ids[0] == 0 and infos[0]["status"] == plc.PLC_E_INVALID
