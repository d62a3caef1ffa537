"""The multicore CPU baseline (OpenMP) against the oracle: the same checks as
the GPU parity tests (p and r within 1e-12, counters, sweep order, cluster),
on R-MAT graphs over mixed alpha, eps and both push rules, and several queries
in a row on one state (the touched-list reset)."""
import numpy as np
import pytest

import synth
from parity import check_query


@pytest.fixture(scope="module")
def cm():
    import cpu_multicore
    cpu_multicore.build(force=False)
    return cpu_multicore


@pytest.mark.parametrize("rule", [0, 1])
def test_multicore_matches_oracle(cm, rule):
    g = synth.rmat(13, 8, seed=3)
    q = synth.batched_queries(g, 24, seed=7, eps_lo=1e-7, eps_hi=1e-4)
    s = cm.Solver(g.off, g.nbr)
    try:
        for i in range(len(q.seeds)):
            res = s.run(int(q.seeds[i]), float(q.alpha[i]), float(q.eps[i]), rule, vectors=True)
            check_query(g, res, int(q.seeds[i]), float(q.alpha[i]), float(q.eps[i]), rule)
    finally:
        s.close()


def test_multicore_hub_and_leaf(cm):
    g = synth.rmat(14, 8, seed=1)
    s = cm.Solver(g.off, g.nbr)
    try:
        for seed in (int(np.argmax(g.deg)), int(np.flatnonzero(g.deg == 1)[0])):
            res = s.run(seed, 0.01, 1e-6, 0, vectors=True)
            check_query(g, res, seed, 0.01, 1e-6, 0)
    finally:
        s.close()


def test_multicore_rejects_bad_input(cm):
    g = synth.rmat(10, 8, seed=2)
    s = cm.Solver(g.off, g.nbr)
    try:
        with pytest.raises(ValueError):
            s.run(g.n, 0.01, 1e-6)
        with pytest.raises(ValueError):
            s.run(0, 1.5, 1e-6)
        iso = np.flatnonzero(g.deg == 0)
        if len(iso):
            with pytest.raises(ValueError):
                s.run(int(iso[0]), 0.01, 1e-6)
    finally:
        s.close()
