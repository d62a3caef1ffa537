"""GPU parity of Nibble (Sec. 3.2, Fig. alg:nibble) on the plain path
against the oracle, through the C ABI: small graphs over (eps, T) including
eps = 1e-300 (the untruncated lazy walk), T = 0, a frontier that empties
early (the previous vector is returned), R-MAT 2^16 with the paper's T = 20,
Nibble interleaved with PR-Nibble and HK-PR on one context, and parameter
checks."""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_hkpr, check_nibble, check_query

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
          "path3": lambda: synth.path(3)}
_cache = {}


def graph(ctx, name):
    if name not in _cache:
        g = GRAPHS[name]()
        _cache[name] = (g, ctx.load_graph(g.off, g.nbr, validate=True))
    return _cache[name]


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("eps,T", [(1e-300, 6), (1e-5, 20), (1e-3, 30), (0.3, 5), (1e-4, 0)])
def test_nibble_matches_oracle(ctx, gname, eps, T):
    g, hg = graph(ctx, gname)
    x = int(np.argmax(g.deg)) if gname not in ("star300", "path3") else (1 if gname == "star300"
                                                                         else 0)
    say("case nibble", gname, "eps", eps, "T", T, "seed", x)
    qid, info = ctx.run_nibble(hg, x, eps, T)
    check_nibble(g, ctx.result(qid, release=True), oracle.nibble(g.off, g.nbr, x, eps, T))


def test_nibble_rmat16_paper_T(ctx):
    g = synth.rmat(16, 8, seed=1)
    hg = ctx.load_graph(g.off, g.nbr)
    for x in synth.uniform_seeds(g, 3, seed=6):
        for eps in (1e-6, 1e-8):
            say("case nibble rmat16 seed", int(x), "eps", eps)
            qid, _ = ctx.run_nibble(hg, int(x), eps, 20)
            out = check_nibble(g, ctx.result(qid, release=True),
                               oracle.nibble(g.off, g.nbr, int(x), eps, 20))
            say("  steps", out["steps"], "support", out["support"])


def test_nibble_rmat20_large_support(ctx):
    """Nibble from the top hub of R-MAT 2^20 (ef 8) with the paper's T = 20
    reaches ~5.5e5 vertices: the sweep's merge sort runs 134 block-sort tiles
    and 8 merge passes with a ragged last tile, and the order, cluster and
    conductance must still match the oracle's."""
    g = synth.rmat(20, 8, seed=3)
    hg = ctx.load_graph(g.off, g.nbr)
    x = int(np.argmax(g.deg))
    say("case nibble rmat20 hub", x, "eps 1e-10 T 20")
    qid, info = ctx.run_nibble(hg, x, 1e-10, 20)
    assert info["support"] > 500000
    out = check_nibble(g, ctx.result(qid, release=True), oracle.nibble(g.off, g.nbr, x, 1e-10, 20))
    say("  steps", out["steps"], "support", out["support"])
    hg.free()


def test_nibble_interleaved_with_prnibble_and_hkpr(ctx):
    g, hg = graph(ctx, "rmat13")
    for x in [int(v) for v in synth.uniform_seeds(g, 2, seed=9)]:
        say("case interleave seed", x)
        qid, _ = ctx.run_nibble(hg, x, 1e-6, 15)
        check_nibble(g, ctx.result(qid, release=True), oracle.nibble(g.off, g.nbr, x, 1e-6, 15))
        ids, _ = ctx.run(hg, [x], 0.01, 1e-6)
        check_query(g, ctx.result(ids[0], release=True), x, 0.01, 1e-6, 0)
        qid, _ = ctx.run_hkpr(hg, x, 10, 1e-5, 4.0)
        check_hkpr(g, ctx.result(qid, release=True), oracle.hkpr(g.off, g.nbr, x, 10, 1e-5, 4.0))


def test_nibble_rejects_bad_parameters(ctx):
    import paper_1604_07515_amd as plc
    g, hg = graph(ctx, "rmat13")
    x = int(np.argmax(g.deg))
    for args in ((x, 0.0, 5), (x, -1.0, 5), (x, 1e-3, -1), (x, 1e-3, 1025), (g.n, 1e-3, 5)):
        with pytest.raises(plc.PlcError) as e:
            ctx.run_nibble(hg, *args)
        assert e.value.code == plc.PLC_E_INVALID
