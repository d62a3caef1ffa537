"""GPU parity of the beta variant of PR-Nibble (end of Sec. 3.3: each
round pushes the top beta fraction of the active set by r/d) against the
oracle, through the C ABI: strict parity where the ranking boundary never
ties, schedule-independent checks (the exact PPR identity with the GPU's
own p and r) where it does, beta 1 equal to the plain path, parameter
checks."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_query, check_same

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1604_07515_amd as plc
    c = plc.Context(arena_bytes=2 << 30)
    yield c
    c.close()


GRAPHS = {"rmat13": lambda: synth.rmat(13, 8, seed=4), "er300": lambda: synth.erdos_renyi(300, 0.03, 7),
          "rmat10": lambda: synth.rmat(10, 8, seed=3), "er1000": lambda: synth.erdos_renyi(1000, 0.01, 3),
          "torus5": lambda: synth.torus3d(5), "path200": lambda: synth.path(200),
          "barbell12": lambda: synth.barbell(12)}
_cache = {}


def graph(ctx, name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, ctx.load_graph(g.off, g.nbr, validate=True))
    return _cache[name]


def beta_oracle(g, x, alpha, eps, beta, rule):
    """The oracle's result, its tie gap widened by the selection gap (a
    near-tie in the ranking may choose a different set under a different
    summation order)."""
    res = oracle.prnibble_beta(g.off, g.nbr, x, alpha, eps, beta, rule)
    return dataclasses.replace(res, min_rel_gap=min(res.min_rel_gap, res.min_sel_gap))


@pytest.mark.parametrize("rule,beta,eps", [(0, 0.2, 1e-4), (0, 0.2, 1e-6), (1, 0.3, 3e-5),
                                           (1, 0.3, 1e-6)])
def test_beta_matches_oracle_strictly(ctx, rule, beta, eps):
    """A graph, fraction and eps whose ranking boundary never ties and whose
    threshold decisions stay clear (oracle gaps > 1e-10 in every round): the
    same rounds, pushes, p and r as the oracle."""
    g, hg = graph(ctx, "er300")
    x = int(np.argmax(g.deg))
    say("case beta strict rule", rule, "beta", beta, "eps", eps)
    qid, _ = ctx.run_beta(hg, x, 0.01, eps, beta, rule)
    out = check_query(g, ctx.result(qid, release=True), x, 0.01, eps, rule,
                      orc=beta_oracle(g, x, 0.01, eps, beta, rule))
    assert not out["tie_push"]


@pytest.mark.parametrize("gname", ["rmat10", "er1000", "torus5", "path200", "barbell12"])
@pytest.mark.parametrize("beta", [0.5, 0.1])
@pytest.mark.parametrize("rule", [0, 1])
def test_beta_schedule_invariants(ctx, gname, beta, rule):
    """Where the ranking boundary ties, a different summation order may pick
    a different set, so the result is checked by what every push schedule
    preserves: the exact PPR identity p = R (chi_x - r) from a dense solve
    with the GPU's own p and r, unit mass, r < eps d everywhere; and the
    oracle's invariants and sweep through check_query."""
    from test_oracle_push import dense_ppr_identity
    g, hg = graph(ctx, gname)
    x = int(np.argmax(g.deg)) if gname != "path200" else 0
    eps = 1e-5
    say("case beta invariants", gname, "beta", beta, "rule", rule)
    qid, _ = ctx.run_beta(hg, x, 0.01, eps, beta, rule)
    res = ctx.result(qid, release=True)
    p, r = res.dense_p(g.n), res.dense_r(g.n)
    p_exact, _ = dense_ppr_identity(g, x, 0.01, r)
    assert np.max(np.abs(p - p_exact)) <= 1e-12 * np.max(p_exact)
    assert abs(p.sum() + r.sum() - 1.0) < 1e-12
    assert np.all(r < eps * np.maximum(g.deg, 1))
    check_query(g, res, x, 0.01, eps, rule, orc=beta_oracle(g, x, 0.01, eps, beta, rule))


def test_beta_rmat16_several_seeds(ctx):
    g = synth.rmat(16, 8, seed=1)
    hg = ctx.load_graph(g.off, g.nbr)
    for x in synth.uniform_seeds(g, 3, seed=7):
        say("case beta rmat16 seed", int(x))
        qid, _ = ctx.run_beta(hg, int(x), 0.01, 1e-6, 0.25)
        check_query(g, ctx.result(qid, release=True), int(x), 0.01, 1e-6, 0,
                    orc=beta_oracle(g, int(x), 0.01, 1e-6, 0.25, 0))


def test_beta_one_is_the_plain_path(ctx):
    g, hg = graph(ctx, "rmat13")
    x = int(np.flatnonzero(g.deg > 2)[11])
    qid, _ = ctx.run_beta(hg, x, 0.01, 1e-6, 1.0)
    ids, _ = ctx.run(hg, [x], 0.01, 1e-6)
    check_same(g, ctx.result(qid, release=True), ctx.result(ids[0], release=True))


def test_beta_rejects_bad_parameters(ctx):
    import paper_1604_07515_amd as plc
    g, hg = graph(ctx, "rmat13")
    for beta in (0.0, -0.1, 1.5):
        with pytest.raises(plc.PlcError) as e:
            ctx.run_beta(hg, 0, 0.01, 1e-6, beta)
        assert e.value.code == plc.PLC_E_INVALID


@pytest.mark.parametrize("rounds,support", [(1, [0]), (2, [0, 1]), (3, [0, 1, 2, 3])])
def test_beta_selection_rule_hand_derived(rounds, support):
    """The hand-derived selection case of the oracle's pins (path 2-1-0-3 with
    leaves 4, 5 on vertex 3; alpha 1/3, eps 1e-3, beta 1/2, seed 0), stopped
    by the round watchdog after 1, 2 and 3 rounds: the GPU picks the
    ceil(beta |S|) largest r/d each round, so p and r equal the derived
    values (round 3 pushes 3 and 2: by r alone it would push 3 and 0, by the
    smallest r/d 0 and 2, and floor would push 3 alone)."""
    import paper_1604_07515_amd as plc
    g = synth.from_edges(6, [(0, 1), (0, 3), (1, 2), (3, 4), (3, 5)])
    want_p = {1: [1 / 2, 0, 0, 0, 0, 0], 2: [1 / 2, 1 / 8, 0, 0, 0, 0],
              3: [1 / 2, 1 / 8, 1 / 32, 1 / 8, 0, 0]}[rounds]
    want_r = {1: [0, 1 / 4, 0, 1 / 4, 0, 0], 2: [1 / 16, 0, 1 / 16, 1 / 4, 0, 0],
              3: [1 / 16 + 1 / 24, 1 / 32, 0, 0, 1 / 24, 1 / 24]}[rounds]
    with plc.Context(arena_bytes=64 << 20, max_rounds=rounds) as c:
        hg = c.load_graph(g.off, g.nbr, validate=True)
        qid, info = c.run_beta(hg, 0, 1.0 / 3.0, 1e-3, 0.5)
        say("case beta hand-derived rounds", rounds, info)
        assert info["status"] == plc.PLC_E_LIMIT and info["rounds"] == rounds
        res = c.result(qid, release=True)
        p, r = res.dense_p(6), res.dense_r(6)
        assert np.flatnonzero(p > 0).tolist() == support
        assert np.allclose(p, want_p, rtol=1e-14, atol=0)
        assert np.allclose(r, want_r, rtol=1e-14, atol=0)
