"""Pins of the HK-PR oracle (Sec. 3.4, Fig. alg:hkpr), CPU only.

  * eps = 1e-300 (nothing is dropped): p equals the polynomial the procedure
    evaluates, sum_{k<N} t^k/k! P^k s + t^(N-1)/(N-1)! P^N s, from dense
    matrix powers (the last level spreads r/d(v) to the neighbours);
  * the level-synchronous oracle equals the sequential queue procedure
    printed in Sec. 3.4 (an independent formulation);
  * a hand-derived threshold case on a 3-vertex path that tells psi_(j+1)
    from psi_j and psi_(j+2);
  * a larger eps drops more: p is monotone in eps, p <= p(eps = 1e-300);
  * a huge eps pushes only the seed; N = 1 spreads the seed's unit once.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def poly(g, x, N, t):
    n = g.n
    P = np.zeros((n, n))
    for v in range(n):
        if g.deg[v] > 0:
            P[g.neighbors(v), v] = 1.0 / g.deg[v]
    s = np.zeros(n)
    s[x] = 1.0
    acc = np.zeros(n)
    vec = s.copy()
    for k in range(N):
        acc += t ** k / math.factorial(k) * vec
        vec = P @ vec
    return acc + t ** (N - 1) / math.factorial(N - 1) * vec


GRAPHS = {"er": lambda: synth.erdos_renyi(40, 0.15, 5), "star": lambda: synth.star(9),
          "path": lambda: synth.path(7), "torus": lambda: synth.torus3d(3),
          "rmat": lambda: synth.rmat(6, 6, seed=2)}


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("N,t", [(1, 1.0), (2, 0.5), (5, 3.0), (12, 10.0)])
def test_tiny_eps_is_the_polynomial(gname, N, t):
    g = GRAPHS[gname]()
    x = int(np.argmax(g.deg))
    res = oracle.hkpr(g.off, g.nbr, x, N, 1e-300, t)
    ref = poly(g, x, N, t)
    assert np.max(np.abs(res.p - ref)) <= 1e-12 * np.max(ref)
    assert res.levels == N


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
@pytest.mark.parametrize("t", [2.0, 5.0])
def test_levels_equal_queue(eps, t):
    g = synth.rmat(9, 8, seed=4)
    x = int(np.flatnonzero(g.deg > 3)[3])
    N = max(1, int(math.ceil(2 * t * math.log(1 / eps))))
    a = oracle.hkpr(g.off, g.nbr, x, N, eps, t)
    b = oracle.hkpr_queue(g.off, g.nbr, x, N, eps, t)
    sup = a.p > 0
    assert np.array_equal(sup, b.p > 0)
    assert np.max(np.abs(a.p[sup] - b.p[sup]) / a.p[sup]) <= 1e-12
    if a.min_rel_gap > 1e-10:
        assert (a.levels, a.pushes, a.edges) == (b.levels, b.pushes, b.edges)


def test_threshold_uses_psi_of_the_next_level():
    """Path 0-1-2, seed 0, N = 2, t = 1: vertex 1 holds r = 1 at level 1 and
    its threshold is e^-1 eps d(1) / (2 N psi_1) with psi_1 = 1 + t/2 = 1.5,
    so it is pushed iff eps <= 3e (~8.15); psi_2 = 1 would move the bound to
    2e and psi_0 = 2.5 to 5e."""
    g = synth.path(3)
    for eps, pushed in ((7.0, True), (9.0, False)):
        res = oracle.hkpr(g.off, g.nbr, 0, 2, eps, 1.0)
        if pushed:
            assert np.allclose(res.p, [1.5, 1.0, 0.5], rtol=0, atol=1e-15) and res.levels == 2
        else:
            assert np.array_equal(res.p, [1.0, 0.0, 0.0]) and res.levels == 1


def test_threshold_psi_at_three_levels():
    """Path 0-1-2, seed 0, N = 3, t = 2: vertex 1 gets r = 2 at level 1, with
    psi_1 = 1 + 2/2 + 4/6 = 8/3, so it is pushed iff eps <= 6 psi_1 e^2 =
    16 e^2 (~118.2); psi_2 = 5/3 would give ~73.9 and psi_0 = 19/3 ~280.8.
    Once pushed, its neighbours get 1 each at level 2, below their threshold
    e^-2 eps / 10 for eps = 100."""
    g = synth.path(3)
    res = oracle.hkpr(g.off, g.nbr, 0, 3, 100.0, 2.0)
    assert np.array_equal(res.p, [1.0, 2.0, 0.0]) and res.levels == 2
    res = oracle.hkpr(g.off, g.nbr, 0, 3, 130.0, 2.0)
    assert np.array_equal(res.p, [1.0, 0.0, 0.0]) and res.levels == 1


def test_monotone_in_eps():
    g = synth.rmat(8, 8, seed=7)
    x = int(np.argmax(g.deg))
    N, t = 12, 4.0
    prev = oracle.hkpr(g.off, g.nbr, x, N, 1e-300, t).p
    for eps in (1e-8, 1e-6, 1e-4, 1e-2, 1.0):
        cur = oracle.hkpr(g.off, g.nbr, x, N, eps, t).p
        assert np.all(cur <= prev * (1 + 1e-12) + 1e-300)
        prev = cur


def test_huge_eps_and_single_level():
    g = synth.star(6)
    res = oracle.hkpr(g.off, g.nbr, 0, 4, 1e6, 2.0)
    assert res.p[0] == 1.0 and np.count_nonzero(res.p) == 1
    res = oracle.hkpr(g.off, g.nbr, 0, 1, 1e-3, 2.0)
    assert res.p[0] == 1.0 and np.allclose(res.p[1:], 1.0 / 6, rtol=0, atol=1e-16)


def test_invalid_inputs():
    g = synth.path(4)
    for args in ((0, 0, 1e-3, 1.0), (-1, 3, 1e-3, 1.0), (0, 3, -1.0, 1.0), (0, 3, 0.0, 1.0),
                 (0, 3, 1e-3, 0.0)):
        with pytest.raises(ValueError):
            oracle.hkpr(g.off, g.nbr, *args)
