"""The parity helper's near-tie blocks (CPU only)."""
import numpy as np

from parity import TIE, tie_blocks


def test_tie_blocks():
    deg = np.ones(6, np.int64)
    p = np.array([6.0, 5.0, 5.0, 4.0, 4.0 * (1 - TIE / 4), 1.0])
    order = np.arange(6)
    blk = tie_blocks(order, p, deg)
    # exact ties (positions 1, 2) stay separate; the near tie (3, 4) is one block
    assert blk.tolist() == [0, 1, 2, 3, 3, 5]
    p2 = np.array([3.0, 3.0, 3.0 * (1 - TIE / 4)])
    assert tie_blocks(np.arange(3), p2, np.ones(3, np.int64)).tolist() == [0, 0, 0]


def test_tie_blocks_other_side():
    deg = np.ones(3, np.int64)
    p = np.array([2.0, 2.0, 1.0])          # exact tie on one side
    q = np.array([2.0, 2.0 * (1 + 1e-15), 1.0])  # a few ulps apart on the other
    assert tie_blocks(np.arange(3), p, deg).tolist() == [0, 1, 2]
    assert tie_blocks(np.arange(3), p, deg, q).tolist() == [0, 0, 2]


def test_cluster_arcs_counts_the_cut():
    import synth
    from parity import cluster_arcs
    g = synth.rmat(9, 8, seed=5)
    rng = np.random.default_rng(0)
    for k in (1, 7, 100, g.n):
        cl = np.sort(rng.choice(g.n, k, replace=False))
        inset = np.zeros(g.n, bool)
        inset[cl] = True
        want = sum(1 for v in cl for w in g.nbr[g.off[v]:g.off[v + 1]] if not inset[w])
        arcs = cluster_arcs(g, cl)
        assert len(arcs) == int(g.deg[cl].sum())
        assert int(np.count_nonzero(~inset[arcs])) == want
