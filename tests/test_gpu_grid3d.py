"""The paper's 3D-grid input at full size: a 215^3 torus (n = 9,938,375,
every vertex of degree 6, 3n edges), alpha 0.01, eps 1e-7, optimized rule --
the setting of the paper's PR-Nibble timings.  The plain path against the
oracle on two seeds (every vertex of a torus is equivalent; the second
query also checks the state reset after the first)."""
import sys

import pytest

import synth
from parity import check_query

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_grid3d_215_full():
    import paper_1604_07515_amd as plc
    g = synth.torus3d(215)
    say("torus 215^3: n", g.n, "arcs", g.arcs)
    with plc.Context(arena_bytes=plc.plain_arena_bytes(g.n, g.arcs) + (256 << 20)) as c:
        hg = c.load_graph(g.off, g.nbr)
        for seed in (0, 4_000_321):
            say("case grid3d seed", seed)
            ids, infos = c.run(hg, [seed], 0.01, 1e-7)
            out = check_query(g, c.result(ids[0], release=True), seed, 0.01, 1e-7, 0)
            say("  rounds", out["rounds"], "support", out["support"], "ties", out["tie_push"],
                out["tie_sweep"])
