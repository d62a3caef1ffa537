"""Comparison of one GPU query against the oracle (shared by the GPU tests).

Tolerances (FP64; the GPU differs from the oracle only in the order of the
atomic additions into r):
  * p and r elementwise within RTOL = 1e-12 relative; zeros must match
    exactly (same support, same nonzero set of r);
  * rounds, pushes, pushed edges, the sweep order, k*, cut and vol exactly;
  * phi exactly (it is cut/den of two equal integers).
When the oracle reports that some filter decision came within TIE = 1e-10
(relative) of its threshold, or that two adjacent sweep keys are within TIE
of each other without being equal, a different summation order may
legitimately flip that decision; such cases are flagged and checked only for
mass, termination and self-consistency of the sweep.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import oracle

RTOL = 1e-12
TIE = 1e-10


def near_tie_in_sweep(order, p, deg) -> bool:
    key = p[order] / deg[order]
    if len(key) < 2:
        return False
    a, b = key[:-1], key[1:]
    close = np.abs(a - b) <= TIE * np.maximum(a, b)
    return bool(np.any(close & (a != b)))


def check_query(g, res, seed, alpha, eps, rule, orc=None, osw=None) -> dict:
    """Assert GPU result `res` (paper_1604_07515_amd.Result) matches the oracle."""
    n = g.n
    deg = g.deg
    info = res.info
    if orc is None:
        orc = oracle.prnibble(g.off, g.nbr, seed, alpha, eps, rule)
    tie_push = orc.min_rel_gap < TIE
    p = res.dense_p(n)
    r = res.dense_r(n)
    # invariants that hold whatever the summation order
    assert abs(p.sum() + r.sum() - 1.0) < 1e-12, "mass"
    assert np.all((r < eps * deg) | (r == 0)), "termination"
    assert info["status"] == 0
    if not tie_push:
        assert info["rounds"] == orc.rounds, (info["rounds"], orc.rounds)
        assert info["pushes"] == orc.pushes
        assert info["edges"] == orc.edges
        sup_o = np.flatnonzero(orc.p > 0)
        sup_g = np.flatnonzero(p > 0)
        assert np.array_equal(sup_o, sup_g), "support"
        assert info["support"] == len(sup_o)
        err = np.abs(p[sup_o] - orc.p[sup_o]) / orc.p[sup_o]
        assert err.max(initial=0) <= RTOL, ("p", err.max())
        nz_o = np.flatnonzero(orc.r != 0)
        nz_g = np.flatnonzero(r != 0)
        assert np.array_equal(nz_o, nz_g), "r nonzeros"
        err_r = np.abs(r[nz_o] - orc.r[nz_o]) / orc.r[nz_o]
        assert err_r.max(initial=0) <= RTOL, ("r", err_r.max())
    # sweep: the GPU's order is the oracle's sweep order of the GPU's own p
    tie_sweep = near_tie_in_sweep(res.sweep_ids, p, deg)
    if osw is None:
        osw = oracle.sweep(g.off, g.nbr, orc.p)
    if not tie_push and not tie_sweep:
        assert np.array_equal(res.sweep_ids, osw.order), "sweep order"
        assert info["kstar"] == osw.kstar
        assert info["cut"] == osw.best_cut and info["vol"] == osw.best_vol
        assert info["phi"] == osw.phi
    # self-consistency: the GPU's reported cut and vol are those of its cluster
    cl = res.cluster
    inset = np.zeros(n, bool)
    inset[cl] = True
    vol = int(deg[cl].sum())
    src = np.repeat(np.arange(n), deg)
    cut = int(np.count_nonzero(inset[src] & ~inset[g.nbr]))
    assert (cut, vol) == (info["cut"], info["vol"])
    den = min(vol, g.arcs - vol)
    assert Fraction(cut, den) == Fraction(info["cut"], den)
    assert info["phi"] == cut / den
    np.testing.assert_array_equal(res.sweep_p, p[res.sweep_ids])
    return {"tie_push": tie_push, "tie_sweep": tie_sweep, "rounds": info["rounds"],
            "edges": info["edges"], "support": info["support"]}
