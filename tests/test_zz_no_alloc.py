"""The allocation-free entry point (plc_run_noalloc) against plc_run.

Two calls in a row through the C ABI, the second on a smaller graph, each
compared with the same query run by plc_run on a context: counters exactly,
p within 1e-12 relative, the sweep order modulo near-tie blocks, the cluster
and conductance; then both against the oracle.  A graph whose working state
exceeds the library's fixed array is refused with PLC_E_NOMEM before any
device work.
"""
import sys

import numpy as np
import pytest

import synth
from parity import check_query, check_same

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc_result(plc, g, seed, alpha, eps, rule):
    import torch
    off = torch.from_numpy(g.off.astype(np.int64)).cuda()
    nbr = torch.from_numpy(g.nbr.astype(np.int32)).cuda()
    rc, info, ids, p = plc.run_noalloc(off, nbr, seed, alpha, eps, rule)
    torch.cuda.synchronize()
    N = info["support"]
    return plc.Result(info, ids[:N].cpu().numpy(), p[:N].cpu().numpy(),
                      np.empty(0, np.int32), np.empty(0, np.float64))


@pytest.mark.parametrize("rule", [0, 1])
def test_noalloc_matches_plc_run_twice(rule):
    import paper_1604_07515_amd as plc
    big = synth.rmat(15, 8, seed=2)
    small = synth.rmat(11, 8, seed=4)
    alpha = 0.01 if rule == 0 else 0.05
    with plc.Context(arena_bytes=1 << 30) as ctx:
        for g, eps in ((big, 1e-7), (small, 1e-6)):
            seed = int(synth.uniform_seeds(g, 1, seed=5)[0])
            say("case noalloc n", g.n, "seed", seed, "rule", rule)
            na = _noalloc_result(plc, g, seed, alpha, eps, rule)
            hg = ctx.load_graph(g.off, g.nbr)
            ids, _ = ctx.run(hg, [seed], alpha, eps, rule)
            ref = ctx.result(ids[0], release=True)
            hg.free()
            for key in ("rounds", "pushes", "edges", "support", "r_nnz", "kstar", "cut", "vol",
                        "phi"):
                assert na.info[key] == ref.info[key], key
            check_same(g, na, ref)
            res = check_query_without_r(g, na, seed, alpha, eps, rule)
            say("  ", res)


def check_query_without_r(g, res, seed, alpha, eps, rule):
    """The oracle comparison of check_query for a result that carries no
    residual vector: p and the sweep (r is compared through plc_run above)."""
    import oracle
    from parity import RTOL, TIE, check_sweep
    orc = oracle.prnibble(g.off, g.nbr, seed, alpha, eps, rule)
    p = res.dense_p(g.n)
    tie = orc.min_rel_gap < TIE
    if not tie:
        assert res.info["rounds"] == orc.rounds and res.info["edges"] == orc.edges
        sup = np.flatnonzero(orc.p > 0)
        assert np.array_equal(sup, np.flatnonzero(p > 0))
        assert np.max(np.abs(p[sup] - orc.p[sup]) / orc.p[sup], initial=0) <= RTOL
    check_sweep(g, res, orc.p, p, tie)
    return {"tie_push": tie, "support": res.info["support"]}


def test_noalloc_refuses_state_larger_than_its_array():
    import torch
    import paper_1604_07515_amd as plc
    off = torch.zeros(4, dtype=torch.int64, device="cuda")
    nbr = torch.zeros(4, dtype=torch.int32, device="cuda")
    q = plc.Context.queries([0], 0.01, 1e-6)
    info = plc.plc_result_info()
    lib = plc.load_library()
    import ctypes as C
    n = 1 << 20  # about 152 MB of state: over the 64 MiB array
    rc = lib.plc_run_noalloc(0, None, n, 4, C.c_void_p(off.data_ptr()), C.c_void_p(nbr.data_ptr()),
                             q, C.c_void_p(off.data_ptr()), C.c_void_p(off.data_ptr()),
                             C.byref(info))
    assert rc == plc.PLC_E_NOMEM
    rc = lib.plc_run_noalloc(0, None, 3, 4, None, C.c_void_p(nbr.data_ptr()), q,
                             C.c_void_p(off.data_ptr()), C.c_void_p(off.data_ptr()), C.byref(info))
    assert rc == plc.PLC_E_INVALID
