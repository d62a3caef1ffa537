"""Pins for the oracle's round-synchronous PR-Nibble (CPU only).

What fixes the answer independently of the oracle's own loops:
  * mass conservation of every push, hence of every round (Sec. 3.3 proof of
    the work theorem);
  * the termination criterion r[v] < eps d(v) (Sec. 3.3, filter);
  * the exact linear-system identity p = R (chi_x - r) with
    R = a' (I - (1 - a') A D^-1)^-1, a' = 2 alpha / (1 + alpha), which every
    push of either rule preserves, checked with a dense solve;
  * the work bound sum_rounds sum_{v in F} d(v) <= (1 - |r|_1) / (a' eps)
    (optimized rule) or / (alpha eps) (original rule) (Sec. 3.3 theorem);
  * closed forms / aggregated recursions on symmetric graphs (K_2, K_n, a
    star seeded at a leaf) that pin the synchronous schedule: every active
    vertex pushes the residual it held at the start of the round;
  * a threshold placed exactly on a residual value, pinning ">=";
  * the barbell: PR-Nibble + sweep returns one clique.
"""
import math

import numpy as np
import pytest

import oracle
import synth

OPT, ORIG = oracle.RULE_OPT, oracle.RULE_ORIG


def consts(rule, alpha):
    if rule == ORIG:
        return alpha, (1.0 - alpha) / 2.0, (1.0 - alpha) / 2.0
    return 2.0 * alpha / (1.0 + alpha), (1.0 - alpha) / (1.0 + alpha), 0.0


def small_graphs():
    gs = [synth.erdos_renyi(80, 0.06, s) for s in range(3)]
    gs += [synth.rmat(10, 8, seed=5), synth.rmat(11, 4, seed=6), synth.barbell(7),
           synth.torus3d(6), synth.star(30), synth.path(40)]
    return gs


def pick_seed(g, i):
    cand = np.flatnonzero(g.deg > 0)
    return int(cand[(37 * i + 11) % len(cand)])


CASES = [(gi, rule, eps) for gi in range(9) for rule in (OPT, ORIG) for eps in (1e-3, 1e-5, 1e-8)]


@pytest.mark.parametrize("gi,rule,eps", CASES)
def test_mass_termination_workbound(gi, rule, eps):
    g = small_graphs()[gi]
    alpha = 0.05 if gi % 2 else 0.01
    x = pick_seed(g, gi)
    res = oracle.prnibble(g.off, g.nbr, x, alpha, eps, rule)
    assert res.status == oracle.OK
    # mass: every push moves mass from r to p and to neighbours' r
    assert abs(res.p.sum() + res.r.sum() - 1.0) < 1e-13
    # termination: no vertex is left with r >= eps d
    # (isolated vertices never receive mass)
    assert np.all((res.r < eps * g.deg.astype(np.float64)) | ((g.deg == 0) & (res.r == 0)))
    assert np.all(res.p >= 0) and np.all(res.r >= 0)
    # work bound
    ap = 2 * alpha / (1 + alpha) if rule == OPT else alpha
    assert ap * eps * res.edges <= res.p.sum() * (1 + 1e-12)
    assert res.pushes == int(res.round_sizes.sum())
    assert res.support == int((res.p > 0).sum())


@pytest.mark.parametrize("rule", [OPT, ORIG])
def test_mass_after_every_round(rule):
    g = synth.rmat(9, 8, seed=9)
    x = pick_seed(g, 3)
    full = oracle.prnibble(g.off, g.nbr, x, 0.02, 1e-6, rule)
    for t in range(1, full.rounds + 1):
        part = oracle.prnibble(g.off, g.nbr, x, 0.02, 1e-6, rule, max_rounds=t)
        assert abs(part.p.sum() + part.r.sum() - 1.0) < 1e-13
        assert part.rounds == t
    # a run stopped early reports LIMIT
    assert oracle.prnibble(g.off, g.nbr, x, 0.02, 1e-6, rule, max_rounds=1).status in (
        oracle.LIMIT, oracle.OK)


def dense_ppr_identity(g, x, alpha, r):
    """p_exact = R (chi_x - r) from a dense solve of the PPR linear system."""
    n = g.n
    A = np.zeros((n, n))
    for v in range(n):
        A[g.neighbors(v), v] = 1.0
    dinv = np.where(g.deg > 0, 1.0 / np.maximum(g.deg, 1), 0.0)
    ap = 2 * alpha / (1 + alpha)
    M = np.eye(n) - (1 - ap) * A * dinv[None, :]
    chi = np.zeros(n)
    chi[x] = 1.0
    return np.linalg.solve(M, ap * (chi - r)), np.linalg.solve(M, ap * chi)


@pytest.mark.parametrize("rule", [OPT, ORIG])
@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-10])
@pytest.mark.parametrize("gname", ["er", "rmat", "barbell", "torus"])
def test_exact_ppr_identity(rule, eps, gname):
    g = {"er": synth.erdos_renyi(90, 0.05, 11), "rmat": synth.rmat(7, 6, seed=12),
         "barbell": synth.barbell(9), "torus": synth.torus3d(4)}[gname]
    lab = synth.components(g)
    x = pick_seed(g, 5)
    keep = lab == lab[x]          # the diffusion never leaves x's component
    idx = np.flatnonzero(keep)
    sub = synth.from_edges(len(idx), [(int(np.searchsorted(idx, v)), int(np.searchsorted(idx, w)))
                                      for v in idx for w in g.neighbors(v) if v < w])
    xs = int(np.searchsorted(idx, x))
    alpha = 0.03
    res = oracle.prnibble(sub.off, sub.nbr, xs, alpha, eps, rule)
    p_exact, p_star = dense_ppr_identity(sub, xs, alpha, res.r)
    assert np.max(np.abs(res.p - p_exact)) <= 1e-12 * np.max(p_exact)
    # |p* - p|_1 = |r|_1 (R is column stochastic) and 0 <= p <= p*
    assert abs(np.abs(p_star - res.p).sum() - res.r.sum()) < 1e-12
    assert np.all(res.p <= p_star + 1e-15)


def test_k2_closed_form():
    alpha, eps = 0.01, 1e-7
    g = synth.path(2)
    res = oracle.prnibble(g.off, g.nbr, 0, alpha, eps, OPT)
    ap = 2 * alpha / (1 + alpha)
    q = 1 - ap
    x = math.log(eps) / math.log(q)
    assert abs(x - round(x)) > 1e-3  # threshold not near a tie
    R = math.floor(x) + 1
    assert R == 806 and res.rounds == R
    p0 = sum(ap * q ** j for j in range(0, R, 2))
    p1 = sum(ap * q ** j for j in range(1, R, 2))
    assert abs(res.p[0] - p0) <= 1e-13 and abs(res.p[1] - p1) <= 1e-13
    assert abs(res.p[0] - 1 / (2 - ap)) < 1e-6
    assert res.round_sizes.tolist() == [1] * R


def kn_recursion(n, alpha, eps, rule):
    """Aggregate two-state simulation of K_n seeded at one vertex."""
    cs, cn, keep = consts(rule, alpha)
    d = n - 1
    a, b, pa, pb = 1.0, 0.0, 0.0, 0.0
    sizes = []
    t = 0
    while True:
        act_a = (t == 0) or a >= eps * d
        act_b = b >= eps * d and b > 0
        if not (act_a or act_b):
            break
        sizes.append(int(act_a) + (n - 1) * int(act_b))
        ra = a if act_a else 0.0
        rb = b if act_b else 0.0
        pa += cs * ra
        pb += cs * rb
        na = (keep * ra if act_a else a) + (cn * rb / d) * (n - 1)
        nb = (keep * rb if act_b else b) + cn * ra / d + (cn * rb / d) * (n - 2)
        a, b = na, nb
        t += 1
    return pa, pb, a, b, sizes


@pytest.mark.parametrize("rule", [OPT, ORIG])
@pytest.mark.parametrize("n,alpha,eps", [(6, 0.01, 1e-4), (12, 0.1, 1e-6), (30, 0.05, 3e-5)])
def test_complete_graph_recursion(rule, n, alpha, eps):
    g = synth.complete(n)
    res = oracle.prnibble(g.off, g.nbr, 0, alpha, eps, rule)
    pa, pb, a, b, sizes = kn_recursion(n, alpha, eps, rule)
    assert res.round_sizes.tolist() == sizes
    assert abs(res.p[0] - pa) <= 1e-13 * pa
    assert np.allclose(res.p[1:], pb, rtol=1e-13, atol=0)
    assert abs(res.r[0] - a) <= 1e-13 * max(a, 1e-300) + 1e-300
    assert np.allclose(res.r[1:], b, rtol=1e-13, atol=1e-300)


def star_leaf_recursion(k, alpha, eps, rule):
    """Three-state simulation of a star (center degree k) seeded at a leaf."""
    cs, cn, keep = consts(rule, alpha)
    s, c, o = 1.0, 0.0, 0.0
    ps = pc = po = 0.0
    sizes = []
    t = 0
    while True:
        act_s = (t == 0) or s >= eps
        act_c = c >= eps * k and c > 0
        act_o = o >= eps and o > 0
        if not (act_s or act_c or act_o):
            break
        sizes.append(int(act_s) + int(act_c) + (k - 1) * int(act_o))
        rs_, rc_, ro_ = (s if act_s else 0.0), (c if act_c else 0.0), (o if act_o else 0.0)
        ps += cs * rs_
        pc += cs * rc_
        po += cs * ro_
        from_c = cn * rc_ / k
        ns = (keep * rs_ if act_s else s) + from_c
        nc = (keep * rc_ if act_c else c) + cn * rs_ / 1 + (cn * ro_ / 1) * (k - 1)
        no = (keep * ro_ if act_o else o) + from_c
        s, c, o = ns, nc, no
        t += 1
    return ps, pc, po, sizes


@pytest.mark.parametrize("rule", [OPT, ORIG])
@pytest.mark.parametrize("k,alpha,eps", [(5, 0.01, 1e-4), (40, 0.05, 1e-6), (200, 0.01, 1e-7)])
def test_star_seeded_at_leaf_recursion(rule, k, alpha, eps):
    g = synth.star(k)
    res = oracle.prnibble(g.off, g.nbr, 1, alpha, eps, rule)
    ps, pc, po, sizes = star_leaf_recursion(k, alpha, eps, rule)
    assert res.round_sizes.tolist() == sizes
    assert abs(res.p[1] - ps) <= 1e-12 * ps
    assert abs(res.p[0] - pc) <= 1e-12 * pc
    if po > 0:
        assert np.allclose(res.p[2:], po, rtol=1e-12, atol=0)


def test_threshold_is_inclusive():
    # Star seeded at its center: each leaf receives c = (cn * 1) / k.  With eps
    # equal to that exact value every leaf sits on the threshold and must push.
    k, alpha = 9, 0.01
    g = synth.star(k)
    cn = (1.0 - alpha) / (1.0 + alpha)
    eps = (cn * 1.0) / float(k)
    res = oracle.prnibble(g.off, g.nbr, 0, alpha, eps, OPT, max_rounds=2)
    assert res.round_sizes.tolist()[:2] == [1, k]


def test_seed_pushed_even_below_threshold():
    g = synth.star(10)
    res = oracle.prnibble(g.off, g.nbr, 0, 0.01, 0.5, OPT)  # eps d(x) = 5 > 1
    assert res.rounds == 1 and res.pushes == 1
    assert res.p[0] == 2 * 0.01 / 1.01


@pytest.mark.parametrize("k", [5, 10, 30])
@pytest.mark.parametrize("alpha,eps", [(0.01, 1e-7), (0.1, 1e-4), (0.01, 1e-3)])
def test_barbell_returns_one_clique(k, alpha, eps):
    g = synth.barbell(k)
    res = oracle.prnibble(g.off, g.nbr, 0, alpha, eps, OPT)
    s = oracle.sweep(g.off, g.nbr, res.p)
    assert sorted(s.cluster.tolist()) == list(range(k))
    assert s.best_cut == 1 and s.best_vol == k * (k - 1) + 1
    assert s.phi == 1.0 / (k * (k - 1) + 1)


def test_invalid_inputs():
    g = synth.from_edges(4, [(0, 1), (1, 2)])  # vertex 3 isolated
    with pytest.raises(ValueError):
        oracle.prnibble(g.off, g.nbr, 3, 0.01, 1e-4)
    for a in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(ValueError):
            oracle.prnibble(g.off, g.nbr, 0, a, 1e-4)
    for e in (0.0, -1e-3, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            oracle.prnibble(g.off, g.nbr, 0, 0.01, e)
    with pytest.raises(ValueError):
        oracle.prnibble(g.off, g.nbr, 7, 0.01, 1e-4)


@pytest.mark.parametrize("rule", [OPT, ORIG])
def test_seed_set_exact_identity(rule):
    """Seed sets (Sec. 3): with the unit mass split equally over the distinct
    seeds, p = R (chi_S / |S| - r) holds exactly (dense solve), mass is
    conserved, and a repeated seed counts once."""
    g = synth.rmat(7, 6, seed=12)
    lab = synth.components(g)
    x = pick_seed(g, 5)
    idx = np.flatnonzero(lab == lab[x])
    sub = synth.from_edges(len(idx), [(int(np.searchsorted(idx, v)), int(np.searchsorted(idx, w)))
                                      for v in idx for w in g.neighbors(v) if v < w])
    seeds = [0, len(idx) // 2, len(idx) - 1]
    alpha = 0.03
    res = oracle.prnibble(sub.off, sub.nbr, seeds + [seeds[0]], alpha, 1e-7, rule)
    n = sub.n
    A = np.zeros((n, n))
    for v in range(n):
        A[sub.neighbors(v), v] = 1.0
    ap = 2 * alpha / (1 + alpha)
    M = np.eye(n) - (1 - ap) * A / np.maximum(sub.deg, 1)[None, :]
    chi = np.zeros(n)
    chi[seeds] = 1.0 / 3.0
    p_exact = np.linalg.solve(M, ap * (chi - res.r))
    assert np.max(np.abs(res.p - p_exact)) <= 1e-12 * np.max(p_exact)
    assert abs(res.p.sum() + res.r.sum() - 1.0) < 1e-12
    again = oracle.prnibble(sub.off, sub.nbr, seeds, alpha, 1e-7, rule)
    assert np.array_equal(again.p, res.p) and np.array_equal(again.r, res.r)
