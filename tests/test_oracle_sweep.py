"""Pins for the oracle's sweep cut (CPU only).

The sweep is pinned by the paper's worked example (Sec. 3.1), by brute force
over every prefix (the definitions of volume, boundary and conductance,
Sec. 2), and by Theorem 1's Z construction, which must agree with both.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _example():
    with open(os.path.join(GOLDEN, "sweep_worked_example.json")) as f:
        fx = json.load(f)
    g = synth.from_edges(fx["n"], fx["edges"])
    return fx, g


def test_worked_example_z_arrays():
    fx, g = _example()
    Z, Zs, Zsum, cuts = oracle.sweep_z(g.off, g.nbr, fx["order"])
    assert Z.tolist() == fx["Z"]
    assert Zs.tolist() == fx["Z_sorted"]
    assert Zsum.tolist() == fx["Z_summed"]
    assert cuts.tolist() == fx["cuts"]


def test_worked_example_sweep():
    fx, g = _example()
    assert g.n == 8 and g.arcs == 16  # n = 8, m = 8
    assert [int(g.deg[v]) for v in fx["order"]] == fx["degrees_by_rank"]
    # Any p whose p/d strictly decreases along A, B, C, D gives that order.
    p = np.zeros(g.n)
    for k, v in enumerate(fx["order"]):
        p[v] = (0.4 - 0.1 * k) * g.deg[v]
    s = oracle.sweep(g.off, g.nbr, p)
    assert s.order.tolist() == fx["order"]
    assert s.vol.tolist() == fx["vol_prefix"]
    assert s.cut.tolist() == fx["cuts"]
    assert s.cluster.tolist() == fx["best_set"]
    assert s.phi == 1.0 / 7.0
    # conductances of the four prefixes: 1, 1/2, 1/7, 3/5 with 2m = 16
    phis = [Fraction(int(c), int(min(v, 16 - v))) for c, v in zip(s.cut, s.vol)]
    assert phis == [Fraction(1), Fraction(1, 2), Fraction(1, 7), Fraction(3, 5)]


def _random_cases():
    cases = []
    for seed in range(6):
        cases.append(synth.erdos_renyi(60, 0.08, seed))
    cases.append(synth.rmat(8, 4, seed=3))
    cases.append(synth.rmat(9, 8, seed=4))
    cases.append(synth.barbell(6))
    cases.append(synth.torus3d(5))
    return cases


@pytest.mark.parametrize("gi", range(10))
def test_sweep_matches_bruteforce_and_z(gi):
    g = _random_cases()[gi]
    rng = np.random.default_rng(100 + gi)
    deg = g.deg
    # Supports with ties in p/d: ratios drawn from a small set of values.
    p = np.where((rng.random(g.n) < 0.6) & (deg > 0),
                 rng.integers(1, 6, g.n) * deg * 0.125, 0.0)
    s = oracle.sweep(g.off, g.nbr, p)
    sup = np.flatnonzero(p > 0)
    assert s.N == len(sup)
    assert sorted(s.order.tolist()) == sup.tolist()
    key = p[s.order] / deg[s.order]
    # non-increasing p/d, equal ratios in ascending id
    for i in range(s.N - 1):
        assert key[i] > key[i + 1] or (key[i] == key[i + 1] and s.order[i] < s.order[i + 1])
    b = oracle.sweep_bruteforce(g.off, g.nbr, s.order)
    assert np.array_equal(b.cut, s.cut) and np.array_equal(b.vol, s.vol)
    assert (b.kstar, b.best_cut, b.best_vol) == (s.kstar, s.best_cut, s.best_vol)
    _, _, _, zc = oracle.sweep_z(g.off, g.nbr, s.order)
    assert np.array_equal(zc, s.cut)
    # vol prefix = inclusive prefix sum of degrees in sweep order
    assert np.array_equal(s.vol, np.cumsum(deg[s.order]))
    # exact argmin, first k on ties, den = 0 excluded
    vt = g.arcs
    best = None
    for k in range(s.N):
        den = min(s.vol[k], vt - s.vol[k])
        if den <= 0:
            continue
        f = Fraction(int(s.cut[k]), int(den))
        if best is None or f < best[0]:
            best = (f, k + 1)
    assert best[1] == s.kstar
    assert s.phi == float(best[0].numerator) / float(best[0].denominator)


def test_sweep_first_index_wins_exact_tie():
    # Three disjoint triangles: prefixes of 3 and 6 vertices both have phi = 0.
    e = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (6, 7), (7, 8), (6, 8)]
    g = synth.from_edges(9, e)
    p = np.array([9, 8, 7, 6, 5, 4, 3, 2, 1], dtype=np.float64)
    s = oracle.sweep(g.off, g.nbr, p)
    assert s.cut.tolist()[2] == 0 and s.cut.tolist()[5] == 0
    assert s.kstar == 3 and s.phi == 0.0


def test_sweep_full_volume_prefix_excluded():
    # The whole K3: the last prefix has vol = 2m, so min(vol, 2m - vol) = 0.
    g = synth.complete(3)
    s = oracle.sweep(g.off, g.nbr, np.array([3.0, 2.0, 1.0]))
    assert s.vol.tolist() == [2, 4, 6]
    assert s.kstar == 1 and s.phi == 1.0


def test_sweep_ties_in_ratio_ascending_id():
    # A star's leaves all get the same p/d; they must come in ascending id.
    g = synth.star(7)
    p = np.full(g.n, 0.01)
    p[0] = 7.0
    s = oracle.sweep(g.off, g.nbr, p)
    assert s.order.tolist() == [0, 1, 2, 3, 4, 5, 6, 7]


def test_sweep_empty_support():
    g = synth.path(5)
    s = oracle.sweep(g.off, g.nbr, np.zeros(5))
    assert s.N == 0 and s.kstar == 0
