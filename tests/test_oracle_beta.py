"""Pins of the beta-variant oracle (PR-Nibble pushing the top beta fraction
of the active set by r/d each round; end of Sec. 3.3), CPU only.

  * beta = 1 is PR-Nibble: the same p and r (to rounding order) and the
    same rounds, pushes and edges;
  * any push schedule keeps the exact PPR identity p = R (chi_x - r) and
    unit mass, and ends with r < eps d everywhere;
  * a tiny beta pushes exactly one vertex (the largest r/d) per round;
  * a hand-derived case fixes the selection rule itself: the key is r/d
    (not r), ranked from the largest (not the smallest), and the round takes
    ceil(beta |S|) vertices (not floor).
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_push import dense_ppr_identity, pick_seed


@pytest.mark.parametrize("rule", [oracle.RULE_OPT, oracle.RULE_ORIG])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_beta_one_is_prnibble(rule, eps):
    g = synth.rmat(10, 8, seed=3)
    x = pick_seed(g, 3)
    a = oracle.prnibble_beta(g.off, g.nbr, x, 0.01, eps, 1.0, rule)
    b = oracle.prnibble(g.off, g.nbr, x, 0.01, eps, rule)
    sup = b.p > 0
    assert np.array_equal(sup, a.p > 0)
    assert np.max(np.abs(a.p[sup] - b.p[sup]) / b.p[sup]) <= 1e-12
    if min(a.min_rel_gap, b.min_rel_gap) > 1e-10:
        assert (a.rounds, a.pushes, a.edges) == (b.rounds, b.pushes, b.edges)


@pytest.mark.parametrize("rule", [oracle.RULE_OPT, oracle.RULE_ORIG])
@pytest.mark.parametrize("beta", [0.05, 0.3, 0.7])
def test_beta_keeps_ppr_identity_and_terminates(rule, beta):
    g = synth.rmat(7, 6, seed=12)
    lab = synth.components(g)
    x = pick_seed(g, 5)
    idx = np.flatnonzero(lab == lab[x])
    sub = synth.from_edges(len(idx), [(int(np.searchsorted(idx, v)), int(np.searchsorted(idx, w)))
                                      for v in idx for w in g.neighbors(v) if v < w])
    xs = int(np.searchsorted(idx, x))
    eps = 1e-6
    res = oracle.prnibble_beta(sub.off, sub.nbr, xs, 0.03, eps, beta, rule)
    p_exact, p_star = dense_ppr_identity(sub, xs, 0.03, res.r)
    assert np.max(np.abs(res.p - p_exact)) <= 1e-12 * np.max(p_exact)
    assert abs(res.p.sum() + res.r.sum() - 1.0) < 1e-12
    assert np.all(res.r < eps * sub.deg)
    assert np.all(res.p <= p_star + 1e-15)


def test_tiny_beta_pushes_one_per_round():
    g = synth.rmat(8, 6, seed=4)
    x = pick_seed(g, 2)
    res = oracle.prnibble_beta(g.off, g.nbr, x, 0.05, 1e-4, 1e-9)
    assert res.pushes == res.rounds > 1


# Hand-derived selection case.  Graph: the path 2 - 1 - 0 - 3 and two leaves
# 4, 5 on vertex 3; degrees d = (2, 2, 1, 3, 1, 1).  Optimized rule with
# alpha = 1/3, so cs = 2a/(1+a) = 1/2 and cn = (1-a)/(1+a) = 1/2; eps = 1e-3,
# beta = 1/2, seed 0.
#   round 1: S = {0}, k = ceil(1/2) = 1: push 0 (rho 1): p0 = 1/2,
#            r1 = r3 = (1/2)(1)/2 = 1/4.
#   round 2: S = {1, 3} with r/d = 1/8, 1/12; k = ceil(1) = 1: push 1 (the
#            largest r/d; the smallest would be 3): p1 = 1/8,
#            r0 = r2 = (1/2)(1/4)/2 = 1/16.
#   round 3: S = {0, 2, 3} with r = 1/16, 1/16, 1/4 and r/d = 1/32, 1/16,
#            1/12; k = ceil(3/2) = 2 (floor would be 1): push 3 and 2 (by r
#            alone 3 and then 0, the tie 0/2 broken by id): p3 = 1/8,
#            p2 = 1/32; 3 sends (1/2)(1/4)/3 = 1/24 to 0, 4, 5 and 2 sends
#            (1/2)(1/16)/1 = 1/32 to 1, so r = (1/16 + 1/24, 1/32, 0, 0, 1/24, 1/24).
_BETA_EDGES = [(0, 1), (0, 3), (1, 2), (3, 4), (3, 5)]


@pytest.mark.parametrize("rounds,support,pushes", [(1, [0], 1), (2, [0, 1], 2),
                                                   (3, [0, 1, 2, 3], 4)])
def test_beta_selection_rule_hand_derived(rounds, support, pushes):
    g = synth.from_edges(6, _BETA_EDGES)
    assert list(g.deg) == [2, 2, 1, 3, 1, 1]
    res = oracle.prnibble_beta(g.off, g.nbr, 0, 1.0 / 3.0, 1e-3, 0.5, max_rounds=rounds)
    assert res.rounds == rounds
    assert res.pushes == pushes
    assert np.flatnonzero(res.p > 0).tolist() == support
    want_p = {1: [1 / 2, 0, 0, 0, 0, 0], 2: [1 / 2, 1 / 8, 0, 0, 0, 0],
              3: [1 / 2, 1 / 8, 1 / 32, 1 / 8, 0, 0]}[rounds]
    want_r = {1: [0, 1 / 4, 0, 1 / 4, 0, 0], 2: [1 / 16, 0, 1 / 16, 1 / 4, 0, 0],
              3: [1 / 16 + 1 / 24, 1 / 32, 0, 0, 1 / 24, 1 / 24]}[rounds]
    assert np.allclose(res.p, want_p, rtol=1e-14, atol=0)
    assert np.allclose(res.r, want_r, rtol=1e-14, atol=0)


def test_beta_invalid():
    g = synth.path(4)
    for beta in (0.0, -0.5, 1.5):
        with pytest.raises(ValueError):
            oracle.prnibble_beta(g.off, g.nbr, 0, 0.01, 1e-4, beta)
