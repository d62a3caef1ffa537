"""GPU parity of the sweep order in every size class of the device sort.

The sweep visits the support in non-increasing p/d (Sec. 3.1).  The device
sort block-sorts 4096-element tiles; when the sweep's bound on the support
is at most 65536 elements one rank-merge launch then places every element
(one to sixteen tiles), above it merge passes double the sorted runs.
PR-Nibble from vertex 0 of the 64^3 torus gives a support in each class, and
the torus's symmetry gives many exactly equal ratios, which the order breaks
by vertex id across tile boundaries.  Each case is compared with the oracle
(order, cluster and conductance; positions whose keys differ by less than
the near-tie bound may swap).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from parity import check_query, tie_blocks

pytestmark = pytest.mark.gpu

OPT = 0
TILE = 4096

# eps, then the support range (lo, hi] that puts the case in its class
CASES = [
    (2e-5, 0, TILE),            # one tile: the block sort alone
    (2e-6, 2 * TILE, 4 * TILE),  # rank merge of four tiles
    (5e-7, 6 * TILE, 8 * TILE),  # rank merge, bound 32768
    (2e-7, 8 * TILE, 10 * TILE),  # rank merge, bound 65536, nine tiles
    (4e-8, 15 * TILE, 16 * TILE),  # rank merge of sixteen tiles
    (2e-8, 16 * TILE, 32 * TILE),  # above 65536: merge passes
]


def own_order(g, res):
    """The sweep order of the GPU's own p: non-increasing p/d (the ratio is
    one IEEE division, the same on both sides), ties by ascending id."""
    ids = res.sweep_ids
    ratio = res.sweep_p / g.deg[ids].astype(np.float64)
    return ids[np.lexsort((ids, -ratio))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torus():
    import paper_1604_07515_amd as plc
    g = synth.torus3d(64)
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20))
    hg = ctx.load_graph(g.off, g.nbr, validate=True)
    yield g, ctx, hg
    ctx.close()


@pytest.mark.parametrize("eps,lo,hi", CASES)
def test_sweep_order_in_each_sort_class(torus, eps, lo, hi):
    g, ctx, hg = torus
    say("case torus64 seed 0 alpha 0.01 eps", eps)
    ids, infos = ctx.run(hg, [0], 0.01, eps, OPT)
    res = ctx.result(ids[0], release=True)
    rep = check_query(g, res, 0, 0.01, eps, OPT)
    say("report", rep)
    assert lo < rep["support"] <= hi
    # the device order is exactly the sort of its own values, position by
    # position (the oracle comparison above lets near-ties swap)
    assert np.array_equal(res.sweep_ids, own_order(g, res))


def test_rmat_supports_of_nine_and_ten_tiles():
    """R-MAT 2^20 (edge factor 16), alpha 0.01, eps 1e-7 from six uniform
    seeds: supports of 32k to 41k, nine or ten block-sort tiles placed by the
    rank merge.  Against the oracle, positions may move only inside runs of
    ratios equal to within the near-tie bound that the two summation orders
    round differently (up to a sixth of them on R-MAT); the order must also be
    exactly the sort of the GPU's own values at every position."""
    import paper_1604_07515_amd as plc
    g = synth.rmat(20, 16, seed=1)
    seeds = [int(s) for s in synth.uniform_seeds(g, 6, seed=5)]
    ctx = plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20))
    try:
        hg = ctx.load_graph(g.off, g.nbr)
        ids, infos = ctx.run(hg, seeds, 0.01, 1e-7, OPT)
        above = 0
        for qid, x in zip(ids, seeds):
            say("case rmat20 seed", x, "alpha 0.01 eps 1e-7")
            res = ctx.result(qid, release=True)
            orc = oracle.prnibble(g.off, g.nbr, x, 0.01, 1e-7, OPT)
            osw = oracle.sweep(g.off, g.nbr, orc.p)
            rep = check_query(g, res, x, 0.01, 1e-7, OPT, orc=orc, osw=osw)
            blk = tie_blocks(osw.order, orc.p, g.deg, res.dense_p(g.n))
            single = np.ones(len(blk), bool)
            single[blk != np.arange(len(blk))] = False
            single[np.unique(blk[blk != np.arange(len(blk))])] = False
            say("report", rep, "strict positions %d of %d" % (single.sum(), len(blk)))
            assert np.array_equal(res.sweep_ids, own_order(g, res))
            if rep["support"] > 8 * TILE:
                above += 1
                assert not rep["tie_push"] and single.mean() >= 0.8
        assert above >= 4
    finally:
        ctx.close()
