"""The support and touched-set bounds behind plc_query_bytes_estimate, checked on
the oracle (CPU): from the push's work bound (Sec. 3.3) every push other than
the seed's moves at least alpha' eps d(v) of the unit mass into p, so at most
1 + 1/(alpha' eps) vertices are pushed and at most 1 + d(seed) + 1/(alpha' eps)
vertices are touched."""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("rule", [oracle.RULE_OPT, oracle.RULE_ORIG])
def test_support_and_touched_bounds(rule):
    g = synth.rmat(11, 8, seed=4)
    rng = np.random.default_rng(7)
    seeds = synth.uniform_seeds(g, 12, seed=9)
    for s in seeds:
        alpha = float(rng.choice([0.01, 0.05, 0.2]))
        eps = float(10 ** rng.uniform(-5, -2))
        res = oracle.prnibble(g.off, g.nbr, int(s), alpha, eps, rule)
        ap = 2 * alpha / (1 + alpha) if rule == oracle.RULE_OPT else alpha
        w = 1.0 / (ap * eps)
        support = int(np.count_nonzero(res.p))
        rnz = int(np.count_nonzero(res.r))
        assert support <= min(g.n, 1 + math.floor(w))
        assert rnz <= min(g.n, 1 + int(g.deg[s]) + math.floor(w))
        # pushed volume outside the seed's first push
        assert res.edges - g.deg[s] <= w * (1 + 1e-12)

