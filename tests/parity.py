"""Comparison of one GPU query against the oracle (shared by the GPU tests).

Tolerances (FP64; the GPU differs from the oracle only in the order of the
atomic additions into r):
  * p and r elementwise within RTOL = 1e-12 relative; zeros must match
    exactly (same support, same nonzero set of r);
  * rounds, pushes, pushed edges, the sweep order, k*, cut and vol exactly;
  * phi exactly (it is cut/den of two equal integers).
When the oracle reports that some filter decision came within TIE = 1e-10
(relative) of its threshold, a different summation order may legitimately
flip that decision; such cases are checked only for mass, termination and
self-consistency of the sweep.  Where adjacent sweep keys of the oracle are
within TIE of each other without being equal (a near-tie block), the GPU may
order that block differently: the orders must then agree as sets block by
block, and k*, cut, vol and phi must agree unless k* falls inside a block.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import oracle

RTOL = 1e-12
TIE = 1e-10


def tie_blocks(order, p, deg, p_other=None):
    """Start index of the near-tie block of every position of a sweep order.

    A run of consecutive positions whose keys p/d differ by at most TIE
    (relative, equal keys included) forms one block that summation order may
    reorder, unless every key of the run is exactly equal both in p and in
    p_other (the other side's values for the same vertices): such runs are
    ordered by ascending id on both sides and stay split into single
    positions.
    """
    key = p[order] / deg[order]
    key2 = None if p_other is None else p_other[order] / deg[order]
    m = len(order)
    start = np.arange(m, dtype=np.int64)
    i = 0
    while i < m:
        j = i
        while j + 1 < m and abs(key[j + 1] - key[j]) <= TIE * max(key[j], key[j + 1]):
            j += 1
        if j > i:
            exact = np.all(key[i:j + 1] == key[i])
            if key2 is not None:
                exact = exact and np.all(key2[i:j + 1] == key2[i])
            if not exact:
                start[i:j + 1] = i
        i = j + 1
    return start


def cluster_arcs(g, cl):
    """Neighbour ids of every arc leaving the vertices of cl (CSR rows concatenated)."""
    cl = np.asarray(cl, np.int64)
    start = g.off[cl].astype(np.int64)
    cnt = (g.off[cl + 1] - g.off[cl]).astype(np.int64)
    base = np.repeat(start - np.concatenate(([0], np.cumsum(cnt)[:-1])), cnt)
    return g.nbr[base + np.arange(int(cnt.sum()), dtype=np.int64)]


def check_query(g, res, seed, alpha, eps, rule, orc=None, osw=None, with_r=True) -> dict:
    """Assert GPU result `res` (paper_1604_07515_amd.Result) matches the oracle.
    with_r=False: the result keeps no residual (PLC_QF_NO_RESIDUAL); p, the
    counters and the sweep are compared, and the residual's nonzero count
    against the oracle's.  The returned dict says whether the oracle flagged
    a near-tie (tie_push: only invariants were then required) and its gap."""
    n = g.n
    deg = g.deg
    info = res.info
    if orc is None:
        orc = oracle.prnibble(g.off, g.nbr, seed, alpha, eps, rule)
    tie_push = orc.min_rel_gap < TIE
    p = res.dense_p(n)
    r = res.dense_r(n)
    # invariants that hold whatever the summation order
    if with_r:
        assert abs(p.sum() + r.sum() - 1.0) < 1e-12, "mass"
        assert np.all((r < eps * deg) | (r == 0)), "termination"
    else:
        assert len(res.r_ids) == 0 and 0.0 < p.sum() <= 1.0 + 1e-12
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
        if with_r:
            nz_g = np.flatnonzero(r != 0)
            assert np.array_equal(nz_o, nz_g), "r nonzeros"
            err_r = np.abs(r[nz_o] - orc.r[nz_o]) / orc.r[nz_o]
            assert err_r.max(initial=0) <= RTOL, ("r", err_r.max())
        else:
            assert info["r_nnz"] == len(nz_o), "r nonzero count"
    tie_sweep = check_sweep(g, res, orc.p, p, tie_push, osw)
    return {"tie_push": tie_push, "gap": orc.min_rel_gap, "tie_sweep": tie_sweep,
            "rounds": info["rounds"], "edges": info["edges"], "support": info["support"]}


def check_sweep(g, res, p_ref, p, tie_push, osw=None) -> bool:
    """The sweep of GPU result `res` (p on the GPU: p) against the oracle's
    sweep of p_ref: order, cluster and conductance equal modulo near-tie
    blocks (positions whose keys differ by < TIE may be swapped), and the
    reported cut and vol recounted from the GPU's own cluster.  Returns
    whether a near-tie block was met."""
    n = g.n
    deg = g.deg
    info = res.info
    if osw is None:
        osw = oracle.sweep(g.off, g.nbr, p_ref)
    tie_sweep = False
    if not tie_push:
        blk = tie_blocks(osw.order, p_ref, deg, p)
        tie_sweep = bool(np.any(blk != np.arange(len(blk))))
        assert len(res.sweep_ids) == len(osw.order), "support size"
        if not tie_sweep:
            assert np.array_equal(res.sweep_ids, osw.order), "sweep order"
        else:
            ends = np.append(np.flatnonzero(np.diff(blk) != 0) + 1, len(blk))
            b0 = 0
            for b1 in ends:
                assert set(res.sweep_ids[b0:b1].tolist()) == set(osw.order[b0:b1].tolist()), \
                    ("sweep order outside a near-tie block", b0, b1)
                b0 = b1
        k = osw.kstar
        inside = tie_sweep and 0 < k < len(blk) and blk[k] == blk[k - 1]
        if not inside:
            assert info["kstar"] == osw.kstar
            assert info["cut"] == osw.best_cut and info["vol"] == osw.best_vol
            assert info["phi"] == osw.phi
    # self-consistency: the GPU's reported cut and vol are those of its cluster
    cl = res.cluster
    inset = np.zeros(n, bool)
    inset[cl] = True
    vol = int(deg[cl].sum())
    cut = int(np.count_nonzero(~inset[cluster_arcs(g, cl)]))
    assert (cut, vol) == (info["cut"], info["vol"])
    den = min(vol, g.arcs - vol)
    assert Fraction(cut, den) == Fraction(info["cut"], den)
    assert info["phi"] == cut / den
    np.testing.assert_array_equal(res.sweep_p, p[res.sweep_ids])
    return tie_sweep


def check_hkpr(g, res, orc) -> dict:
    """GPU HK-PR result `res` against the oracle's level-synchronous HK-PR
    `orc` (oracle.hkpr): p within RTOL with the same support, levels,
    pushes and edges exactly, no residual reported, and the sweep as for
    PR-Nibble.  Near-threshold decisions (oracle gap < TIE) may flip under a
    different summation order: then only the sweep's self-consistency and
    the bound p <= p(eps = 0) are left to the caller."""
    info = res.info
    p = res.dense_p(g.n)
    assert info["status"] == 0 and info["r_nnz"] == 0
    tie_push = orc.min_rel_gap < TIE
    if not tie_push:
        assert (info["rounds"], info["pushes"], info["edges"]) == (orc.levels, orc.pushes,
                                                                   orc.edges)
        sup = orc.p > 0
        assert np.array_equal(sup, p > 0), "support"
        assert info["support"] == int(sup.sum())
        err = np.abs(p[sup] - orc.p[sup]) / orc.p[sup]
        assert err.max(initial=0) <= RTOL, ("p", err.max())
    tie_sweep = check_sweep(g, res, orc.p, p, tie_push)
    return {"tie_push": tie_push, "tie_sweep": tie_sweep, "levels": info["rounds"],
            "support": info["support"]}


def check_same(g, a, b) -> None:
    """Two GPU results of the same query (e.g. alone and inside a batch) agree:
    counters exactly, p within RTOL, the sweep order modulo near-tie blocks,
    and the cluster unless k* falls inside such a block."""
    deg = g.deg
    for key in ("rounds", "pushes", "edges", "support", "r_nnz"):
        assert a.info[key] == b.info[key], key
    pa, pb = a.dense_p(g.n), b.dense_p(g.n)
    sup = np.flatnonzero(pa > 0)
    assert np.array_equal(sup, np.flatnonzero(pb > 0))
    assert np.max(np.abs(pa[sup] - pb[sup]) / pa[sup], initial=0) <= RTOL
    blk = tie_blocks(a.sweep_ids, pa, deg, pb)
    ends = np.append(np.flatnonzero(np.diff(blk) != 0) + 1, len(blk))
    b0 = 0
    for b1 in ends:
        assert set(a.sweep_ids[b0:b1].tolist()) == set(b.sweep_ids[b0:b1].tolist())
        b0 = b1
    k = a.info["kstar"]
    if not (0 < k < len(blk) and blk[k] == blk[k - 1]):
        for key in ("kstar", "cut", "vol", "phi"):
            assert a.info[key] == b.info[key], key


def check_properties(g, res, eps, with_r=True):
    """Invariants of one result that need no oracle run."""
    info = res.info
    assert info["status"] == 0
    assert info["support"] == len(res.sweep_ids) == len(res.sweep_p)
    assert np.all(res.sweep_p > 0)
    if with_r:
        assert abs(res.sweep_p.sum() + res.r_vals.sum() - 1.0) < 1e-12, "mass"
        assert np.all(res.r_vals < eps * g.deg[res.r_ids]), "termination"
    else:
        assert len(res.r_ids) == 0 and res.sweep_p.sum() <= 1.0 + 1e-12
    key = res.sweep_p / g.deg[res.sweep_ids]
    assert np.all(key[1:] <= key[:-1] * (1 + 1e-10)), "sweep order"
    cl = res.cluster
    inset = np.zeros(g.n, bool)
    inset[cl] = True
    assert info["vol"] == int(g.deg[cl].sum())
    assert info["cut"] == int(np.count_nonzero(~inset[cluster_arcs(g, cl)]))
    assert info["phi"] == info["cut"] / min(info["vol"], g.arcs - info["vol"])


def check_nibble(g, res, orc, rtol=RTOL) -> dict:
    """GPU Nibble result against the oracle's (oracle.nibble): the returned
    vector within rtol (RTOL, or a per-vertex array) with the same support,
    steps, pushes and edges exactly, no residual reported, and the sweep as
    for PR-Nibble; near threshold decisions (oracle gap < TIE) relax the
    first part."""
    info = res.info
    p = res.dense_p(g.n)
    assert info["status"] == 0 and info["r_nnz"] == 0
    tie_push = orc.min_rel_gap < TIE
    if not tie_push:
        assert (info["rounds"], info["pushes"], info["edges"]) == (orc.iterations, orc.pushes,
                                                                   orc.edges)
        sup = orc.p > 0
        assert np.array_equal(sup, p > 0), "support"
        err = np.abs(p[sup] - orc.p[sup]) / orc.p[sup]
        tol = rtol[sup] if np.ndim(rtol) else rtol
        assert np.all(err <= tol), ("p", err.max(), float(np.max(err / tol)))
    tie_sweep = check_sweep(g, res, orc.p, p, tie_push)
    return {"tie_push": tie_push, "tie_sweep": tie_sweep, "steps": info["rounds"],
            "support": info["support"]}
