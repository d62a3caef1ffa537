"""Python binding of libplc: parallel local graph clustering on MI355X (gfx950).

Argument marshalling only.  Every step of PR-Nibble and the sweep cut runs in
the HIP kernels of ``libplc.so``; this module passes pointers and sizes
through the C ABI of ``include/plc.h``.  PyTorch supplies the device arena
(one uint8 tensor) and the stream.  If the library has not been built, or no
GPU is present, the calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplc.so")

PLC_OK = 0
PLC_E_INVALID = -1
PLC_E_NOMEM = -2
PLC_E_BUSY = -3
PLC_E_NOTREADY = -4
PLC_E_NOTFOUND = -5
PLC_E_LIMIT = -6
PLC_E_HIP = -7
PLC_RULE_OPT = 0
PLC_RULE_ORIG = 1
PLC_GRAPH_VALIDATE = 1
PLC_LAUNCH_GRAPH = 0
PLC_LAUNCH_DIRECT = 1
PLC_STATE_DENSE = 0
PLC_STATE_COMPACT = 1
PLC_QF_NO_RESIDUAL = 1

# Every symbol include/plc.h declares.
SYMBOLS = ("plc_status_str", "plc_init", "plc_destroy", "plc_graph_load", "plc_graph_free",
           "plc_graph_info_get", "plc_run", "plc_run_set", "plc_run_hkpr", "plc_run_nibble",
           "plc_run_beta", "plc_run_noalloc",
           "plc_result_info_get",
           "plc_result_copy", "plc_result_copy_many",
           "plc_release", "plc_arena_free_bytes", "plc_timing_enable", "plc_timing_get",
           "plc_batch_reserve", "plc_submit", "plc_progress", "plc_poll", "plc_wait",
           "plc_query_bytes_estimate", "plc_run_batched", "plc_autotune")


class PlcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s: %s (%d)" % (what, status_str(code), code))
        self.code = code


class plc_options(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("batch_slots", C.c_int32),
                ("launch_mode", C.c_int32), ("batch_state", C.c_int32),
                ("bin_min_edges", C.c_int32), ("reserved", C.c_int32 * 3)]


class plc_query(C.Structure):
    _fields_ = [("seed", C.c_int32), ("rule", C.c_uint32), ("alpha", C.c_double),
                ("eps", C.c_double), ("flags", C.c_uint32), ("reserved", C.c_uint32)]


class plc_graph_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("arcs", C.c_int64), ("max_degree", C.c_int64),
                ("bytes", C.c_int64)]


class plc_result_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32), ("pushes", C.c_int64),
                ("edges", C.c_int64), ("support", C.c_int64), ("kstar", C.c_int64),
                ("cut", C.c_int64), ("vol", C.c_int64), ("phi", C.c_double),
                ("r_nnz", C.c_int64), ("launches", C.c_int32), ("loop_rounds", C.c_int32),
                ("loop_edges", C.c_int64), ("host_ns", C.c_int64),
                ("device_ns", C.c_int64), ("bin_rounds", C.c_int32), ("flags", C.c_uint32),
                ("bin_edges", C.c_int64), ("pipelined", C.c_int32), ("table_grows", C.c_int32),
                ("table_cap", C.c_int64), ("pull_rounds", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in self.names()}

    @classmethod
    def names(cls) -> list:
        """Field names of the info dict (the reserved word left out)."""
        return [k for k, _ in cls._fields_ if k != "reserved"]


PLC_TUNE_PLAIN = 1
PLC_TUNE_BATCH = 2


class plc_tune(C.Structure):
    _fields_ = [("plain_self", C.c_int32), ("plain_scatter", C.c_int32),
                ("plain_sweep", C.c_int32), ("batch_self", C.c_int32),
                ("batch_scatter", C.c_int32), ("batch_sweep", C.c_int32),
                ("plain_ms", C.c_double), ("batch_ms", C.c_double),
                ("candidates", C.c_int32), ("plain_bin_min_edges", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class plc_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("units", C.c_int64),
                ("entries", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libplc.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libplc.so is not built (run __graft_entry__.build() or "
                          "python paper_1604_07515_amd/build.py)")
    import torch  # noqa: F401  -- loads the HIP runtime torch was built with
    lib = C.CDLL(path)
    P, I32, I64, U32, U64, D, SZ = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64,
                                    C.c_double, C.c_size_t)
    sig = {
        "plc_status_str": ([I32], C.c_char_p),
        "plc_init": ([C.POINTER(P), I32, P, SZ, P, C.POINTER(plc_options)], I32),
        "plc_destroy": ([P], I32),
        "plc_graph_load": ([P, I64, I64, P, I32, P, U32, C.POINTER(P)], I32),
        "plc_graph_free": ([P, P], I32),
        "plc_graph_info_get": ([P, C.POINTER(plc_graph_info)], I32),
        "plc_run": ([P, P, C.POINTER(plc_query), I32, C.POINTER(U64),
                     C.POINTER(plc_result_info)], I32),
        "plc_run_set": ([P, P, P, I32, C.c_double, C.c_double, I32, C.POINTER(U64),
                         C.POINTER(plc_result_info)], I32),
        "plc_run_noalloc": ([I32, P, I64, I64, P, P, C.POINTER(plc_query), P, P,
                             C.POINTER(plc_result_info)], I32),
        "plc_run_hkpr": ([P, P, I32, I32, C.c_double, C.c_double, C.POINTER(U64),
                          C.POINTER(plc_result_info)], I32),
        "plc_run_nibble": ([P, P, I32, C.c_double, I32, C.POINTER(U64),
                            C.POINTER(plc_result_info)], I32),
        "plc_run_beta": ([P, P, C.POINTER(plc_query), C.c_double, C.POINTER(U64),
                          C.POINTER(plc_result_info)], I32),
        "plc_result_info_get": ([P, U64, C.POINTER(plc_result_info)], I32),
        "plc_result_copy": ([P, U64, P, P, P, P], I32),
        "plc_result_copy_many": ([P, I32, P, P, P, P, P], I32),
        "plc_release": ([P, U64], I32),
        "plc_arena_free_bytes": ([P, C.POINTER(SZ), C.POINTER(SZ)], I32),
        "plc_timing_enable": ([P, I32], I32),
        "plc_timing_get": ([P, C.POINTER(plc_kernel_time), C.POINTER(plc_kernel_time),
                            C.POINTER(plc_kernel_time)], I32),
        "plc_batch_reserve": ([P, P, I32, C.POINTER(I32)], I32),
        "plc_submit": ([P, P, C.POINTER(plc_query), I32, C.POINTER(U64)], I32),
        "plc_progress": ([P, P, C.POINTER(I32), C.POINTER(U64), I32, C.POINTER(I32)], I32),
        "plc_poll": ([P, U64, C.POINTER(I32)], I32),
        "plc_wait": ([P, U64, I64], I32),
        "plc_query_bytes_estimate": ([P, C.POINTER(plc_query)], SZ),
        "plc_run_batched": ([P, P, C.POINTER(plc_query), I32, C.POINTER(U64),
                             C.POINTER(plc_result_info)], I32),
        "plc_autotune": ([P, P, C.POINTER(plc_query), I32, I32, C.POINTER(plc_tune)], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_str(code: int) -> str:
    try:
        return load_library().plc_status_str(code).decode()
    except ImportError:
        return "status %d" % code


def _check(code: int, what: str) -> int:
    if code != PLC_OK:
        raise PlcError(code, what)
    return code


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def _parts(counts, dtype):
    """Host arrays for one kind of vector of several results (one array per
    result, as a lone result gets) and their addresses (0 for an empty one)."""
    views = [np.empty(int(c), dtype) for c in counts]
    ptrs = np.fromiter((v.__array_interface__["data"][0] if len(v) else 0 for v in views),
                       np.uint64, len(views))
    return ptrs, views


@dataclass
class Result:
    """Vectors of a finished query (host copies)."""
    info: dict
    sweep_ids: np.ndarray   # support in sweep order
    sweep_p: np.ndarray     # p at those vertices
    r_ids: np.ndarray       # nonzeros of r (unspecified order)
    r_vals: np.ndarray

    @property
    def cluster(self) -> np.ndarray:
        return self.sweep_ids[: self.info["kstar"]]

    def dense_p(self, n: int) -> np.ndarray:
        p = np.zeros(n)
        p[self.sweep_ids] = self.sweep_p
        return p

    def dense_r(self, n: int) -> np.ndarray:
        r = np.zeros(n)
        r[self.r_ids] = self.r_vals
        return r


class Graph:
    def __init__(self, ctx: "Context", handle: C.c_void_p, n: int, arcs: int):
        self.ctx, self.handle, self.n, self.arcs = ctx, handle, n, arcs

    def info(self) -> dict:
        gi = plc_graph_info()
        _check(self.ctx.lib.plc_graph_info_get(self.handle, C.byref(gi)), "plc_graph_info_get")
        return {k: getattr(gi, k) for k, _ in gi._fields_}

    def free(self):
        if self.handle:
            _check(self.ctx.lib.plc_graph_free(self.ctx.handle, self.handle), "plc_graph_free")
            self.handle = None


class Context:
    """A libplc context on one GPU, with a torch-owned arena and stream."""

    def __init__(self, arena_bytes: int, device: int = 0, stream=None, max_rounds: int = 0,
                 graphs: bool = True, compact: bool = False, bin_min_edges: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libplc needs a GPU; torch.cuda.is_available() is False")
        self.lib = load_library()
        self.device = device
        self.arena_bytes = int(arena_bytes)
        dev = torch.device("cuda", device)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=dev)
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        opt = plc_options()
        opt.max_rounds = max_rounds
        opt.launch_mode = PLC_LAUNCH_GRAPH if graphs else PLC_LAUNCH_DIRECT
        opt.batch_state = PLC_STATE_COMPACT if compact else PLC_STATE_DENSE
        opt.bin_min_edges = int(bin_min_edges)
        h = C.c_void_p()
        _check(self.lib.plc_init(C.byref(h), device, C.c_void_p(aligned), int(arena_bytes),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(opt)), "plc_init")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.plc_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load_graph(self, off: np.ndarray, nbr: np.ndarray, validate: bool = False) -> Graph:
        """Copy a CSR graph into the arena.  int32 offsets are passed as such
        (32-bit CSR), anything else as int64."""
        bits = 32 if np.asarray(off).dtype == np.int32 else 64
        off = np.ascontiguousarray(off, dtype=np.int32 if bits == 32 else np.int64)
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        n = len(off) - 1
        h = C.c_void_p()
        _check(self.lib.plc_graph_load(self.handle, n, len(nbr), _ptr(off), bits, _ptr(nbr),
                                       PLC_GRAPH_VALIDATE if validate else 0, C.byref(h)),
               "plc_graph_load")
        return Graph(self, h, n, len(nbr))

    @staticmethod
    def queries(seeds, alpha, eps, rule=PLC_RULE_OPT, flags=0):
        if isinstance(seeds, (int, np.integer)):
            seeds = (seeds,)
        if isinstance(seeds, (list, tuple)) and all(np.isscalar(x) for x in (alpha, eps, rule)):
            # one parameter set for all seeds: no array broadcasting
            qa = (plc_query * len(seeds))()
            a, e, r, f = float(alpha), float(eps), int(rule), int(flags)
            for i, s in enumerate(seeds):
                q = qa[i]
                q.seed = int(s)
                q.rule = r
                q.alpha = a
                q.eps = e
                q.flags = f
            return qa
        seeds = np.atleast_1d(np.asarray(seeds, dtype=np.int64))
        k = len(seeds)
        alpha = np.broadcast_to(np.asarray(alpha, np.float64), (k,))
        eps = np.broadcast_to(np.asarray(eps, np.float64), (k,))
        rule = np.broadcast_to(np.asarray(rule, np.int64), (k,))
        qa = (plc_query * k)()
        for i in range(k):
            qa[i].seed = int(seeds[i])
            qa[i].rule = int(rule[i])
            qa[i].alpha = float(alpha[i])
            qa[i].eps = float(eps[i])
            qa[i].flags = int(flags)
        return qa

    def run(self, g: Graph, seeds, alpha, eps, rule=PLC_RULE_OPT, check: bool = True,
                flags: int = 0):
        """Plain path: queries one after another.  Returns (ids, infos)."""
        qa = self.queries(seeds, alpha, eps, rule, flags)
        k = len(qa)
        ids = (C.c_uint64 * k)()
        infos = (plc_result_info * k)()
        rc = self.lib.plc_run(self.handle, g.handle, qa, k, ids, infos)
        if check and rc not in (PLC_OK,):
            raise PlcError(rc, "plc_run")
        return list(ids), [x.as_dict() for x in infos]

    def run_set(self, g: Graph, seeds, alpha, eps, rule=PLC_RULE_OPT, check: bool = True):
        """Plain path from a seed set (unit mass split equally over the
        distinct seeds).  Returns (id, info)."""
        sv = np.ascontiguousarray(np.atleast_1d(np.asarray(seeds)), dtype=np.int32)
        qid = C.c_uint64()
        info = plc_result_info()
        rc = self.lib.plc_run_set(self.handle, g.handle, _ptr(sv), len(sv), float(alpha),
                                  float(eps), int(rule), C.byref(qid), C.byref(info))
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_run_set")
        return qid.value, info.as_dict()

    def run_hkpr(self, g: Graph, seed: int, N: int, eps: float, t: float, check: bool = True):
        """Plain path: deterministic heat-kernel PageRank (Taylor degree N)
        from seed, then the sweep cut.  Returns (id, info)."""
        qid = C.c_uint64()
        info = plc_result_info()
        rc = self.lib.plc_run_hkpr(self.handle, g.handle, int(seed), int(N), float(eps), float(t),
                                   C.byref(qid), C.byref(info))
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_run_hkpr")
        return qid.value, info.as_dict()

    def run_nibble(self, g: Graph, seed: int, eps: float, T: int, check: bool = True):
        """Plain path: Nibble (truncated lazy walk, at most T steps) from
        seed, then the sweep cut.  Returns (id, info)."""
        qid = C.c_uint64()
        info = plc_result_info()
        rc = self.lib.plc_run_nibble(self.handle, g.handle, int(seed), float(eps), int(T),
                                     C.byref(qid), C.byref(info))
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_run_nibble")
        return qid.value, info.as_dict()

    def run_beta(self, g: Graph, seed: int, alpha: float, eps: float, beta: float,
                 rule=PLC_RULE_OPT, check: bool = True):
        """Plain path: PR-Nibble pushing the top beta fraction of the active
        set by r/d each round.  Returns (id, info)."""
        qa = self.queries([int(seed)], alpha, eps, rule)
        qid = C.c_uint64()
        info = plc_result_info()
        rc = self.lib.plc_run_beta(self.handle, g.handle, qa, float(beta), C.byref(qid),
                                   C.byref(info))
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_run_beta")
        return qid.value, info.as_dict()

    # ---- batched path
    def batch_reserve(self, g: Graph, slots: int) -> int:
        got = C.c_int32()
        _check(self.lib.plc_batch_reserve(self.handle, g.handle, int(slots), C.byref(got)),
               "plc_batch_reserve")
        return got.value

    def submit(self, g: Graph, seeds, alpha, eps, rule=PLC_RULE_OPT, check: bool = True,
                   flags: int = 0):
        qa = self.queries(seeds, alpha, eps, rule, flags)
        ids = (C.c_uint64 * len(qa))()
        rc = self.lib.plc_submit(self.handle, g.handle, qa, len(qa), ids)
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_submit")
        return list(ids)

    def progress(self, g: Graph, finished: list | None = None) -> int:
        """One global step of the batch engine; returns queries still queued or
        running.  Ids of queries that finished in the step are appended to
        `finished` when a list is given."""
        left = C.c_int32()
        nd = C.c_int32()
        cap = 1024
        buf = (C.c_uint64 * cap)()
        _check(self.lib.plc_progress(self.handle, g.handle, C.byref(left), buf, cap, C.byref(nd)),
               "plc_progress")
        if finished is not None:
            finished.extend(buf[i] for i in range(min(nd.value, cap)))
        return left.value

    def poll(self, qid: int) -> bool:
        done = C.c_int32()
        _check(self.lib.plc_poll(self.handle, qid, C.byref(done)), "plc_poll")
        return bool(done.value)

    def wait(self, qid: int, timeout_us: int = -1) -> bool:
        """Step the query's batch engine until it has finished; False on timeout."""
        rc = self.lib.plc_wait(self.handle, qid, int(timeout_us))
        if rc == PLC_E_NOTREADY:
            return False
        _check(rc, "plc_wait")
        return True

    def query_bytes_estimate(self, g: Graph, seed: int, alpha: float, eps: float,
                             rule: int = PLC_RULE_OPT) -> int:
        """Arena bytes one query occupies on the batch engine (slot state + result bound)."""
        qa = self.queries([seed], alpha, eps, rule)
        return int(self.lib.plc_query_bytes_estimate(g.handle, qa))

    def run_batched(self, g: Graph, seeds, alpha, eps, rule=PLC_RULE_OPT, check: bool = True,
                        flags: int = 0):
        """Batched path: submit all and step until every query has finished."""
        qa = self.queries(seeds, alpha, eps, rule, flags)
        k = len(qa)
        ids = (C.c_uint64 * k)()
        infos = (plc_result_info * k)()
        rc = self.lib.plc_run_batched(self.handle, g.handle, qa, k, ids, infos)
        if check and rc != PLC_OK:
            raise PlcError(rc, "plc_run_batched")
        return list(ids), [x.as_dict() for x in infos]

    def autotune(self, g: Graph, seeds, alpha, eps, which: int, rule=PLC_RULE_OPT) -> dict:
        """Pick launch shapes for graph g from a sample of queries (results discarded)."""
        qa = self.queries(seeds, alpha, eps, rule)
        out = plc_tune()
        _check(self.lib.plc_autotune(self.handle, g.handle, qa, len(qa), which, C.byref(out)),
               "plc_autotune")
        return out.as_dict()

    def result_info(self, qid: int) -> dict:
        info = plc_result_info()
        _check(self.lib.plc_result_info_get(self.handle, qid, C.byref(info)), "plc_result_info_get")
        return info.as_dict()

    def result(self, qid: int, release: bool = False) -> Result:
        info = plc_result_info()
        _check(self.lib.plc_result_info_get(self.handle, qid, C.byref(info)), "plc_result_info_get")
        N, R = info.support, info.r_nnz
        if info.flags & PLC_QF_NO_RESIDUAL:
            R = 0  # the result keeps no residual vector
        ids = np.empty(N, np.int32)
        p = np.empty(N, np.float64)
        rid = np.empty(R, np.int32)
        rv = np.empty(R, np.float64)
        _check(self.lib.plc_result_copy(self.handle, qid, _ptr(ids), _ptr(p), _ptr(rid), _ptr(rv)),
               "plc_result_copy")
        if release:
            self.release(qid)
        return Result(info.as_dict(), ids, p, rid, rv)

    def results(self, qids, release: bool = False) -> list:
        """result() for several finished queries with one GPU round trip
        (plc_result_copy_many)."""
        qids = [int(q) for q in qids]
        if not qids:
            return []
        k = len(qids)
        arr = (plc_result_info * k)()
        for j, qid in enumerate(qids):
            _check(self.lib.plc_result_info_get(self.handle, qid, C.byref(arr[j])),
                   "plc_result_info_get")
        rec = np.frombuffer(arr, dtype=np.dtype(plc_result_info))
        n = rec["support"].astype(np.int64)
        # a result that keeps no residual vector has no r parts
        nr = np.where(rec["flags"] & PLC_QF_NO_RESIDUAL, 0, rec["r_nnz"]).astype(np.int64)
        names = plc_result_info.names()
        infos = [dict(zip(names, row)) for row in rec[names].tolist()]
        parts = [_parts(n, np.int32), _parts(n, np.float64), _parts(nr, np.int32),
                 _parts(nr, np.float64)]
        ids = np.asarray(qids, np.uint64)
        _check(self.lib.plc_result_copy_many(self.handle, k, _ptr(ids),
                                             *[ptrs.ctypes.data for ptrs, _ in parts]),
               "plc_result_copy_many")
        if release:
            for qid in qids:
                self.release(qid)
        return [Result(info, *(views[j] for _, views in parts)) for j, info in enumerate(infos)]

    def release(self, qid: int):
        _check(self.lib.plc_release(self.handle, qid), "plc_release")

    def arena_free(self):
        t, l = C.c_size_t(), C.c_size_t()
        _check(self.lib.plc_arena_free_bytes(self.handle, C.byref(t), C.byref(l)), "plc_arena_free")
        return t.value, l.value

    def timing(self, on: bool):
        _check(self.lib.plc_timing_enable(self.handle, int(on)), "plc_timing_enable")

    def timing_get(self) -> dict:
        a, b, c = plc_kernel_time(), plc_kernel_time(), plc_kernel_time()
        _check(self.lib.plc_timing_get(self.handle, C.byref(a), C.byref(b), C.byref(c)),
               "plc_timing_get")
        return {"scatter": a.as_dict(), "self": b.as_dict(), "sweep": c.as_dict()}


def batch_arena_bytes(n: int, arcs: int, slots: int, compact: bool = False,
                      table_bytes: int = 0) -> int:
    """Arena bytes for a batch engine with `slots` slots (on top of the plain path).

    Dense layout: the slots' per-vertex state (40 B per vertex per slot).
    Compact layout: `table_bytes` for the running queries' tables (36 B per
    table record; plc_query_bytes_estimate bounds one query's need)."""
    per_slot = 0 if compact else 40 * n
    nf_cap = min(max(2 * n, 1 << 22), slots * n)
    nf_cap = max(nf_cap, n)
    e_cap = max(2 * arcs, 1 << 26)
    s_cap = max(min(2 * n, slots * n), n)
    fixed = (28 * nf_cap + 4 * (e_cap // 1024 + 2) + 96 * (max(nf_cap, s_cap) // 1024 + 2)
             + 56 * s_cap + 1024 * slots + 8 * n + (1 << 20))
    return int((per_slot * slots + fixed) * 17 // 16 + (192 << 20) + table_bytes)


def run_noalloc(off, nbr, seed: int, alpha: float, eps: float, rule: int = PLC_RULE_OPT,
                flags: int = 0, device: int = 0, stream=None, out=None, check: bool = True):
    """plc_run_noalloc (one plain query, working state in the library's fixed
    device array, nothing allocated by the library).  off, nbr: torch tensors
    on the GPU (int64 n+1, int32 arcs).  out: optional (ids, p) torch tensors
    of n entries on the same GPU, else allocated here.  Returns (status,
    info, ids, p) with ids[:support], p[:support] the sweep order and p."""
    import torch
    lib = load_library()
    n = int(off.numel()) - 1
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=off.device),
               torch.empty(n, dtype=torch.float64, device=off.device))
    ids, p = out
    st = stream if stream is not None else torch.cuda.current_stream(off.device)
    q = Context.queries([int(seed)], alpha, eps, rule, flags)
    info = plc_result_info()
    rc = lib.plc_run_noalloc(int(device), C.c_void_p(st.cuda_stream), n, int(nbr.numel()),
                             C.c_void_p(off.data_ptr()), C.c_void_p(nbr.data_ptr()), q,
                             C.c_void_p(ids.data_ptr()), C.c_void_p(p.data_ptr()), C.byref(info))
    if check and rc != PLC_OK:
        raise PlcError(rc, "plc_run_noalloc")
    return rc, info.as_dict(), ids, p


def plain_arena_bytes(n: int, arcs: int) -> int:
    """Arena bytes the plain path needs for one graph, plus 64 MiB for results."""
    per_vertex = 168          # offsets, state records, frontier, sweep and HK-PR buffers
    per_arc = 4               # neighbour ids
    tiles = 4 * (arcs // 1024 + 2)
    scans = 3 * 16 * (n // 1024 + 2) + 24 * (n // 1024 + 2)
    # binned scatter (graphs up to 6,291,456 vertices): pairs (8 B per edge of the
    # largest binned round, at most 2^23), the per-chunk run table (2049
    # ints per 2048-edge chunk) and the pull records (16 B per vertex)
    binned = n <= 1536 * 4096
    chunks = (min(max(arcs, 1), 1 << 23) + 2047) // 2048 if binned else 0
    bins = n // 16 + 12 * 2048 + chunks * (8 * 2048 + 4 * 2049) + 7 * 256
    bins += 16 * n if binned else 0
    return int(per_vertex * (n + 1) + per_arc * arcs + tiles + scans + bins + (64 << 20)
               + 8 * 1025 + 2048)
