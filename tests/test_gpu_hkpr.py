"""GPU parity of deterministic HK-PR (Sec. 3.4, Fig. alg:hkpr) on the plain
path against the oracle's level-synchronous HK-PR, through the C ABI:
small graphs over (N, eps, t) including eps = 1e-300 (nothing is dropped:
the whole Taylor polynomial) and N = 1, an R-MAT graph with the practical N = 2 t log(1/eps),
HK-PR and PR-Nibble queries interleaved on one context (state reset between
algorithms), and parameter checks."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hkpr, check_query

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


GRAPHS = {"rmat13": lambda: synth.rmat(13, 8, seed=4), "torus12": lambda: synth.torus3d(12),
          "barbell12": lambda: synth.barbell(12), "star300": lambda: synth.star(300),
          "k40": lambda: synth.complete(40)}
_cache = {}


def graph(ctx, name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, ctx.load_graph(g.off, g.nbr, validate=True))
    return _cache[name]


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("N,eps,t", [(1, 1e-3, 1.0), (6, 1e-300, 2.0), (8, 1e-4, 3.0),
                                     (20, 1e-6, 5.0)])
def test_hkpr_matches_oracle(ctx, gname, N, eps, t):
    g, hg = graph(ctx, gname)
    x = int(np.argmax(g.deg)) if gname != "star300" else 1
    say("case hkpr", gname, "N", N, "eps", eps, "t", t, "seed", x)
    qid, info = ctx.run_hkpr(hg, x, N, eps, t)
    orc = oracle.hkpr(g.off, g.nbr, x, N, eps, t)
    check_hkpr(g, ctx.result(qid, release=True), orc)


@pytest.mark.parametrize("t,eps", [(3.0, 1e-4), (10.0, 1e-5)])
def test_hkpr_rmat16_practical_N(ctx, t, eps):
    g = synth.rmat(16, 8, seed=1)
    hg = ctx.load_graph(g.off, g.nbr)
    N = int(math.ceil(2 * t * math.log(1 / eps)))
    for x in synth.uniform_seeds(g, 3, seed=5):
        say("case hkpr rmat16 t", t, "eps", eps, "N", N, "seed", int(x))
        qid, info = ctx.run_hkpr(hg, int(x), N, eps, t)
        out = check_hkpr(g, ctx.result(qid, release=True), oracle.hkpr(g.off, g.nbr, int(x), N,
                                                                       eps, t))
        say("  levels", out["levels"], "support", out["support"])


def test_hkpr_and_prnibble_interleaved(ctx):
    g, hg = graph(ctx, "rmat13")
    xs = [int(x) for x in synth.uniform_seeds(g, 3, seed=8)]
    for x in xs:
        say("case interleave seed", x)
        qid, _ = ctx.run_hkpr(hg, x, 10, 1e-5, 4.0)
        check_hkpr(g, ctx.result(qid, release=True), oracle.hkpr(g.off, g.nbr, x, 10, 1e-5, 4.0))
        ids, _ = ctx.run(hg, [x], 0.01, 1e-6)
        check_query(g, ctx.result(ids[0], release=True), x, 0.01, 1e-6, 0)


def test_hkpr_rejects_bad_parameters(ctx):
    import paper_1604_07515_amd as plc
    g, hg = graph(ctx, "rmat13")
    x = int(np.argmax(g.deg))
    for args in ((x, 0, 1e-3, 1.0), (x, 1025, 1e-3, 1.0), (x, 4, -1e-3, 1.0), (x, 4, 0.0, 1.0),
                 (x, 4, 1e-3, 0.0),
                 (g.n, 4, 1e-3, 1.0), (-1, 4, 1e-3, 1.0)):
        with pytest.raises(plc.PlcError) as e:
            ctx.run_hkpr(hg, *args)
        assert e.value.code == plc.PLC_E_INVALID
