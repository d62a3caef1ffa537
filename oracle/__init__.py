"""CPU oracle for round-synchronous PR-Nibble and the sweep cut.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only code that may import this
package.  The product path (``paper_1604_07515_amd``) never imports it, and the
two share no code.

The arithmetic lives in ``oracle.c`` (plain C, binary64, no FMA contraction);
this module only compiles it with gcc and marshals numpy arrays through ctypes.
Every function takes a graph as CSR arrays: ``off`` (int64, n+1) and ``nbr``
(int32, off[n]), undirected, each edge stored as two arcs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RULE_OPT = 0   # optimized push rule, Sec. 3.3 "An Optimization"
RULE_ORIG = 1  # original push rule, Sec. 3.3 / Fig. alg:pr-nibble

OK, E_INVALID, E_NOMEM, LIMIT = 0, -1, -2, 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, binary64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _PushStats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("pushes", C.c_int64), ("edges", C.c_int64),
                ("support", C.c_int64), ("min_rel_gap", C.c_double),
                ("max_frontier", C.c_int32), ("status", C.c_int32)]


class _SweepResult(C.Structure):
    _fields_ = [("N", C.c_int64), ("kstar", C.c_int64), ("cut", C.c_int64),
                ("vol", C.c_int64), ("den", C.c_int64), ("phi", C.c_double),
                ("vol_total", C.c_int64)]


class _HkStats(C.Structure):
    _fields_ = [("levels", C.c_int64), ("pushes", C.c_int64), ("edges", C.c_int64),
                ("support", C.c_int64), ("min_rel_gap", C.c_double)]


class _NbStats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("pushes", C.c_int64), ("edges", C.c_int64),
                ("support", C.c_int64), ("min_rel_gap", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.oracle_prnibble.argtypes = [C.c_int64, P, P, P, C.c_int32, C.c_double, C.c_double,
                                        C.c_int32, C.c_int64, P, P, P, C.POINTER(_PushStats)]
        lib.oracle_prnibble.restype = C.c_int
        lib.oracle_sweep_order.argtypes = [C.c_int64, P, P, P]
        lib.oracle_sweep_order.restype = C.c_int64
        lib.oracle_sweep.argtypes = [C.c_int64, P, P, P, P, P, P, C.POINTER(_SweepResult)]
        lib.oracle_sweep.restype = C.c_int
        lib.oracle_sweep_bruteforce.argtypes = [C.c_int64, P, P, P, C.c_int64, P, P,
                                                C.POINTER(_SweepResult)]
        lib.oracle_sweep_bruteforce.restype = C.c_int
        lib.oracle_sweep_z.argtypes = [C.c_int64, P, P, P, C.c_int64, P, P, P, P, P, P]
        lib.oracle_sweep_z.restype = C.c_int
        lib.oracle_prnibble_beta.argtypes = [C.c_int64, P, P, C.c_int32, C.c_double, C.c_double,
                                             C.c_int32, C.c_double, C.c_int64, P, P,
                                             C.POINTER(_PushStats), C.POINTER(C.c_double)]
        lib.oracle_prnibble_beta.restype = C.c_int
        lib.oracle_nibble.argtypes = [C.c_int64, P, P, C.c_int32, C.c_double, C.c_int32, P,
                                      C.POINTER(_NbStats)]
        lib.oracle_nibble.restype = C.c_int
        for fn in (lib.oracle_hkpr, lib.oracle_hkpr_queue):
            fn.argtypes = [C.c_int64, P, P, C.c_int32, C.c_int32, C.c_double, C.c_double, P,
                           C.POINTER(_HkStats)]
            fn.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(off, nbr):
    off = np.ascontiguousarray(off, dtype=np.int64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    return off, nbr, len(off) - 1


@dataclass
class PushResult:
    p: np.ndarray          # dense float64, length n
    r: np.ndarray          # dense float64, length n
    rounds: int
    pushes: int
    edges: int             # sum over rounds of sum_{v in F} d(v)
    support: int
    min_rel_gap: float     # closest approach of any filter decision to its threshold
    max_frontier: int
    status: int            # OK or LIMIT
    round_sizes: np.ndarray


def prnibble(off, nbr, seeds, alpha: float, eps: float, rule: int = RULE_OPT,
             max_rounds: int = 1 << 30) -> PushResult:
    """Round-synchronous PR-Nibble (Sec. 3.3, Figs. alg:pr-nibble / alg:pr-nibble2)."""
    off, nbr, n = _csr(off, nbr)
    seeds = np.atleast_1d(np.asarray(seeds, dtype=np.int32))
    p = np.zeros(n, np.float64)
    r = np.zeros(n, np.float64)
    cap = int(min(max_rounds, 1 << 20))
    rs = np.zeros(cap, np.int32)
    st = _PushStats()
    rc = _load().oracle_prnibble(n, _ptr(off), _ptr(nbr), _ptr(seeds), len(seeds), alpha, eps,
                                 rule, min(max_rounds, cap), _ptr(p), _ptr(r), _ptr(rs),
                                 C.byref(st))
    if rc < 0:
        raise ValueError("oracle_prnibble rejected its input (code %d)" % rc)
    return PushResult(p, r, st.rounds, st.pushes, st.edges, st.support, st.min_rel_gap,
                      st.max_frontier, rc, rs[: st.rounds].copy())


@dataclass
class SweepResult:
    order: np.ndarray      # ordered support v_1..v_N
    cut: np.ndarray        # |boundary(S_k)|, k = 1..N
    vol: np.ndarray        # vol(S_k)
    N: int
    kstar: int             # best prefix length (cluster = order[:kstar])
    best_cut: int
    best_vol: int
    best_den: int
    phi: float
    vol_total: int

    @property
    def cluster(self) -> np.ndarray:
        return self.order[: self.kstar]


def _sweep_result(order, cut, vol, res) -> SweepResult:
    return SweepResult(order, cut, vol, res.N, res.kstar, res.cut, res.vol, res.den, res.phi,
                       res.vol_total)


def sweep_order(off, nbr, p) -> np.ndarray:
    """Support of p sorted by non-increasing p/d, ties by ascending id (Sec. 3.1)."""
    off, nbr, n = _csr(off, nbr)
    p = np.ascontiguousarray(p, dtype=np.float64)
    order = np.zeros(n, np.int32)
    N = _load().oracle_sweep_order(n, _ptr(off), _ptr(p), _ptr(order))
    if N < 0:
        raise ValueError("oracle_sweep_order rejected its input (code %d)" % N)
    return order[:N].copy()


def sweep(off, nbr, p) -> SweepResult:
    """Sequential sweep cut (Sec. 3.1), exact rational argmin, first k on ties."""
    off, nbr, n = _csr(off, nbr)
    p = np.ascontiguousarray(p, dtype=np.float64)
    order = np.zeros(n, np.int32)
    cut = np.zeros(n, np.int64)
    vol = np.zeros(n, np.int64)
    res = _SweepResult()
    rc = _load().oracle_sweep(n, _ptr(off), _ptr(nbr), _ptr(p), _ptr(order), _ptr(cut),
                              _ptr(vol), C.byref(res))
    if rc < 0:
        raise ValueError("oracle_sweep rejected its input (code %d)" % rc)
    N = res.N
    return _sweep_result(order[:N].copy(), cut[:N].copy(), vol[:N].copy(), res)


def sweep_bruteforce(off, nbr, order) -> SweepResult:
    """Every prefix recounted from the definitions of vol and boundary (Sec. 2)."""
    off, nbr, n = _csr(off, nbr)
    order = np.ascontiguousarray(order, dtype=np.int32)
    N = len(order)
    cut = np.zeros(max(N, 1), np.int64)
    vol = np.zeros(max(N, 1), np.int64)
    res = _SweepResult()
    rc = _load().oracle_sweep_bruteforce(n, _ptr(off), _ptr(nbr), _ptr(order), N, _ptr(cut),
                                         _ptr(vol), C.byref(res))
    if rc < 0:
        raise ValueError("oracle_sweep_bruteforce failed (code %d)" % rc)
    return _sweep_result(order.copy(), cut[:N].copy(), vol[:N].copy(), res)


def sweep_z(off, nbr, order):
    """Theorem 1's Z-array construction; returns (Z, Z_sorted, Z_summed, cuts).

    Z and Z_sorted are (first, second) pair arrays; Z_summed is the inclusive
    prefix sum of Z_sorted's first values paired with its second values.
    """
    off, nbr, n = _csr(off, nbr)
    order = np.ascontiguousarray(order, dtype=np.int32)
    N = len(order)
    vol = int(sum(off[v + 1] - off[v] for v in order))
    L = max(2 * vol, 1)
    zf = np.zeros(L, np.int32); zs = np.zeros(L, np.int64)
    zfs = np.zeros(L, np.int32); zss = np.zeros(L, np.int64)
    zsum = np.zeros(L, np.int64); cut = np.zeros(max(N, 1), np.int64)
    ln = _load().oracle_sweep_z(n, _ptr(off), _ptr(nbr), _ptr(order), N, _ptr(zf), _ptr(zs),
                                _ptr(zfs), _ptr(zss), _ptr(zsum), _ptr(cut))
    if ln < 0:
        raise ValueError("oracle_sweep_z failed (code %d)" % ln)
    Z = np.stack([zf[:ln], zs[:ln]], 1)
    Zs = np.stack([zfs[:ln], zss[:ln]], 1)
    Zsum = np.stack([zsum[:ln], zss[:ln]], 1)
    return Z, Zs, Zsum, cut[:N].copy()


@dataclass
class HkResult:
    p: np.ndarray          # dense float64, length n
    levels: int            # levels processed (the last pushes into p)
    pushes: int            # (vertex, level) entries processed
    edges: int             # sum of d(v) over processed entries
    support: int
    min_rel_gap: float     # closest approach of a threshold decision to its threshold


def _hk(fn, off, nbr, seed, N, eps, t) -> HkResult:
    off, nbr, n = _csr(off, nbr)
    p = np.zeros(n, np.float64)
    st = _HkStats()
    rc = fn(n, _ptr(off), _ptr(nbr), int(seed), int(N), float(eps), float(t), _ptr(p), C.byref(st))
    if rc < 0:
        raise ValueError("HK-PR oracle rejected its input (code %d)" % rc)
    return HkResult(p, st.levels, st.pushes, st.edges, st.support, st.min_rel_gap)


def hkpr(off, nbr, seed, N: int, eps: float, t: float) -> HkResult:
    """Deterministic HK-PR, level-synchronous (Sec. 3.4, Fig. alg:hkpr)."""
    return _hk(_load().oracle_hkpr, off, nbr, seed, N, eps, t)


def hkpr_queue(off, nbr, seed, N: int, eps: float, t: float) -> HkResult:
    """Deterministic HK-PR, the sequential queue procedure of Sec. 3.4
    (dense (N+1) x n residual table: small graphs only)."""
    return _hk(_load().oracle_hkpr_queue, off, nbr, seed, N, eps, t)


@dataclass
class NibbleResult:
    p: np.ndarray          # the returned vector, dense float64
    iterations: int        # iterations whose next vector was computed
    pushes: int
    edges: int
    support: int
    min_rel_gap: float


def nibble(off, nbr, seed, eps: float, T: int) -> NibbleResult:
    """Nibble, the truncated lazy random walk (Sec. 3.2, Fig. alg:nibble)."""
    off, nbr, n = _csr(off, nbr)
    p = np.zeros(n, np.float64)
    st = _NbStats()
    rc = _load().oracle_nibble(n, _ptr(off), _ptr(nbr), int(seed), float(eps), int(T), _ptr(p),
                               C.byref(st))
    if rc < 0:
        raise ValueError("oracle_nibble rejected its input (code %d)" % rc)
    return NibbleResult(p, st.iterations, st.pushes, st.edges, st.support, st.min_rel_gap)


@dataclass
class BetaResult:
    p: np.ndarray
    r: np.ndarray
    rounds: int
    pushes: int
    edges: int
    support: int
    min_rel_gap: float     # closest approach of a threshold decision to its threshold
    min_sel_gap: float     # closest relative gap between the last chosen and first unchosen key
    status: int


def prnibble_beta(off, nbr, seed, alpha: float, eps: float, beta: float, rule: int = RULE_OPT,
                  max_rounds: int = 1 << 30) -> BetaResult:
    """PR-Nibble pushing only the top beta fraction of the active set by r/d
    each round (end of Sec. 3.3)."""
    off, nbr, n = _csr(off, nbr)
    p = np.zeros(n, np.float64)
    r = np.zeros(n, np.float64)
    st = _PushStats()
    gap = C.c_double()
    rc = _load().oracle_prnibble_beta(n, _ptr(off), _ptr(nbr), int(seed), float(alpha), float(eps),
                                      int(rule), float(beta), int(max_rounds), _ptr(p), _ptr(r),
                                      C.byref(st), C.byref(gap))
    if rc < 0:
        raise ValueError("oracle_prnibble_beta rejected its input (code %d)" % rc)
    return BetaResult(p, r, st.rounds, st.pushes, st.edges, st.support, st.min_rel_gap, gap.value,
                      rc)
