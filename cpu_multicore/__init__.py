"""Multicore CPU PR-Nibble + sweep cut (OpenMP), a measurement baseline.

The paper's shared-memory algorithm (Sec. 3.3 round-synchronous push, Sec. 3.1
sweep) run on the host's cores: the benchmark reports its throughput beside
the GPU's.  It is neither the oracle nor the product path and shares no code
with either; the tests check it against the oracle like any other
implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prnibble_omp.c")
_LIB = os.path.join(_HERE, "libcmc.so")


def build(force: bool = True) -> str:
    """Compile prnibble_omp.c into libcmc.so (gcc -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Res(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("pushes", C.c_int64), ("edges", C.c_int64),
                ("support", C.c_int64), ("kstar", C.c_int64), ("cut", C.c_int64),
                ("vol", C.c_int64), ("phi", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.cmc_create.argtypes = [C.c_int64]
        lib.cmc_create.restype = P
        lib.cmc_destroy.argtypes = [P]
        lib.cmc_run.argtypes = [P, P, P, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                C.c_int32, C.POINTER(_Res)]
        lib.cmc_run.restype = C.c_int
        lib.cmc_vectors.argtypes = [P, P, P, P]
        lib.cmc_threads.restype = C.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the runs use (OMP_NUM_THREADS, else the host's cores)."""
    return int(_load().cmc_threads())


class Result:
    """One finished query, with the attributes the GPU binding's results have."""

    def __init__(self, info, p, r, order):
        self.info = info
        self._p, self._r = p, r
        self.sweep_ids = order
        self.sweep_p = p[order]
        self.r_ids = np.flatnonzero(r != 0).astype(np.int32)
        self.r_vals = r[self.r_ids]

    def dense_p(self, n):
        return self._p

    def dense_r(self, n):
        return self._r

    @property
    def cluster(self):
        return self.sweep_ids[: self.info["kstar"]]


class Solver:
    """Dense per-graph state; queries run one after another, each on all threads."""

    def __init__(self, off, nbr):
        self.off = np.ascontiguousarray(off, dtype=np.int64)
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        self.n = len(self.off) - 1
        self._s = _load().cmc_create(self.n)
        if not self._s:
            raise MemoryError("cmc_create: out of host memory")

    def close(self):
        if self._s:
            _load().cmc_destroy(self._s)
            self._s = None

    def __del__(self):
        self.close()

    def run(self, seed, alpha, eps, rule=0, max_rounds=1 << 30, vectors=False):
        res = _Res()
        rc = _load().cmc_run(self._s, self.off.ctypes.data, self.nbr.ctypes.data, int(seed),
                             float(alpha), float(eps), int(rule), int(min(max_rounds, 2**31 - 1)),
                             C.byref(res))
        if rc != 0:
            raise ValueError("cmc_run rejected its input (code %d)" % rc)
        info = {"status": 0, "rounds": res.rounds, "pushes": res.pushes, "edges": res.edges,
                "support": res.support, "kstar": res.kstar, "cut": res.cut, "vol": res.vol,
                "phi": res.phi}
        if not vectors:
            return info
        p = np.zeros(self.n, np.float64)
        r = np.zeros(self.n, np.float64)
        order = np.zeros(max(res.support, 1), np.int32)
        _load().cmc_vectors(self._s, p.ctypes.data, r.ctypes.data, order.ctypes.data)
        info["r_nnz"] = int(np.count_nonzero(r))
        return Result(info, p, r, order[: res.support].copy())
