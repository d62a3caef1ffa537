"""Pins of the Nibble oracle (Sec. 3.2, Fig. alg:nibble), CPU only.

  * eps = 1e-300 (nothing is truncated): p_T is the lazy random walk
    W^T e_x, W = (I + A D^-1) / 2, from dense matrix powers, and keeps
    unit mass;
  * hand-derived cases on the path 0-1-2 that pin the inclusive threshold
    (p'(v) >= eps d(v)), the dropping of mass outside the frontier, and the
    rule that an empty frontier returns the previous vector;
  * T = 0 returns the seed's indicator.
"""
import numpy as np
import pytest

import oracle
import synth


def lazy_walk(g, x, T):
    n = g.n
    W = 0.5 * np.eye(n)
    for v in range(n):
        if g.deg[v] > 0:
            W[g.neighbors(v), v] += 0.5 / g.deg[v]
    p = np.zeros(n)
    p[x] = 1.0
    for _ in range(T):
        p = W @ p
    return p


GRAPHS = {"er": lambda: synth.erdos_renyi(40, 0.15, 5), "star": lambda: synth.star(9),
          "path": lambda: synth.path(7), "torus": lambda: synth.torus3d(3),
          "rmat": lambda: synth.rmat(6, 6, seed=2), "barbell": lambda: synth.barbell(6)}


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("T", [1, 2, 7, 20])
def test_tiny_eps_is_the_lazy_walk(gname, T):
    g = GRAPHS[gname]()
    x = int(np.argmax(g.deg))
    res = oracle.nibble(g.off, g.nbr, x, 1e-300, T)
    ref = lazy_walk(g, x, T)
    assert np.max(np.abs(res.p - ref)) <= 1e-12 * np.max(ref)
    assert abs(res.p.sum() - 1.0) < 1e-12
    assert res.iterations == T


def test_path_threshold_and_return_rule():
    g = synth.path(3)
    # eps 0.3: p1 = (1/2, 1/2, 0); only 0 passes (0.5 >= 0.3, 0.5 < 0.6).
    # p2 keeps only vertex 0's mass: (1/4, 1/4, 0), nobody passes -> p1.
    res = oracle.nibble(g.off, g.nbr, 0, 0.3, 5)
    assert np.array_equal(res.p, [0.5, 0.5, 0.0]) and res.iterations == 2
    # eps 0.5: 0.5 >= 0.5 passes (inclusive) -> same outcome
    res = oracle.nibble(g.off, g.nbr, 0, 0.5, 5)
    assert np.array_equal(res.p, [0.5, 0.5, 0.0]) and res.iterations == 2
    # eps 0.6: nobody passes after the first step -> the seed's indicator
    res = oracle.nibble(g.off, g.nbr, 0, 0.6, 5)
    assert np.array_equal(res.p, [1.0, 0.0, 0.0]) and res.iterations == 1
    # T = 1 stops with p1 whatever the frontier
    res = oracle.nibble(g.off, g.nbr, 0, 0.3, 1)
    assert np.array_equal(res.p, [0.5, 0.5, 0.0]) and res.iterations == 1


def test_zero_iterations_and_invalid():
    g = synth.star(5)
    res = oracle.nibble(g.off, g.nbr, 0, 1e-3, 0)
    assert res.p[0] == 1.0 and np.count_nonzero(res.p) == 1 and res.iterations == 0
    for args in ((-1, 1e-3, 3), (0, 0.0, 3), (0, 1e-3, -1)):
        with pytest.raises(ValueError):
            oracle.nibble(g.off, g.nbr, *args)
