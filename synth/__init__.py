"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module generates graphs and query parameters only; it contains none of
the clustering method's arithmetic, and it imports neither the oracle nor the
product package.

Graphs are undirected and unweighted, stored as CSR: ``off`` int64 (n+1) and
``nbr`` int32 (off[n]); each undirected edge appears as two arcs, adjacency
lists are sorted ascending, with no self-loops or duplicates.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from collections import deque
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "libsynth.so")

# R-MAT quadrant probabilities used for every synthetic power-law graph here.
RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        lib.synth_rmat.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_double, C.c_double,
                                   C.c_uint64, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]
        lib.synth_rmat.restype = C.c_int64
        lib.synth_free.argtypes = [C.c_void_p]
        lib.synth_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        _lib = lib
    return _lib


@dataclass
class Graph:
    off: np.ndarray  # int64, n+1
    nbr: np.ndarray  # int32, 2m
    name: str = ""

    @property
    def n(self) -> int:
        return len(self.off) - 1

    @property
    def arcs(self) -> int:
        return int(self.off[-1])

    @property
    def deg(self) -> np.ndarray:
        return np.diff(self.off)

    def neighbors(self, v: int) -> np.ndarray:
        return self.nbr[self.off[v]: self.off[v + 1]]


def from_edges(n: int, edges, name: str = "") -> Graph:
    """CSR from an undirected edge list (symmetrised, deduplicated, sorted)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]], 0)
    key = np.unique(both[:, 0] * n + both[:, 1])
    src = (key // n).astype(np.int64)
    dst = (key % n).astype(np.int32)
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return Graph(off, dst, name)


def rmat(scale: int, edge_factor: int, seed: int = 1, abcd=RMAT_ABCD) -> Graph:
    """Undirected R-MAT graph, 2^scale vertices, edge_factor * 2^scale samples.

    No vertex relabelling is applied, so vertex 0 is the highest-degree hub.
    """
    a, b, c, _ = abcd
    lib = _load()
    po, pn = C.c_void_p(), C.c_void_p()
    ns = edge_factor << scale
    arcs = lib.synth_rmat(scale, ns, a, b, c, seed, C.byref(po), C.byref(pn))
    if arcs < 0:
        raise MemoryError("synth_rmat failed")
    n = 1 << scale
    off = np.empty(n + 1, np.int64)
    nbr = np.empty(arcs, np.int32)
    lib.synth_copy(off.ctypes.data, po, off.nbytes)
    lib.synth_copy(nbr.ctypes.data, pn, nbr.nbytes)
    lib.synth_free(po)
    lib.synth_free(pn)
    return Graph(off, nbr, "rmat%d_ef%d_s%d" % (scale, edge_factor, seed))


def validate(g: Graph) -> None:
    """Raise if g is not a simple undirected CSR graph with sorted rows."""
    off, nbr, n = g.off, g.nbr, g.n
    if off[0] != 0 or np.any(np.diff(off) < 0) or off[-1] != len(nbr):
        raise ValueError("bad offsets")
    if len(nbr) and (nbr.min() < 0 or nbr.max() >= n):
        raise ValueError("neighbour id out of range")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    if np.any(src == nbr):
        raise ValueError("self-loop")
    key = src * n + nbr
    if len(key) > 1 and np.any(np.diff(key) <= 0):
        raise ValueError("rows not strictly ascending (unsorted or duplicate)")
    rev = nbr.astype(np.int64) * n + src
    if not np.array_equal(np.sort(rev), key):
        raise ValueError("not symmetric")


def components(g: Graph) -> np.ndarray:
    """Connected-component label per vertex (labels = smallest id in the component)."""
    n = g.n
    lab = np.full(n, -1, np.int64)
    off, nbr = g.off, g.nbr
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s
        q = deque([s])
        while q:
            v = q.popleft()
            for w in nbr[off[v]: off[v + 1]]:
                if lab[w] < 0:
                    lab[w] = s
                    q.append(w)
    return lab


def largest_component_min_vertex(g: Graph) -> int:
    """Smallest vertex id of the largest connected component."""
    lab = components(g)
    ids, counts = np.unique(lab, return_counts=True)
    best = ids[counts == counts.max()].min()
    return int(best)


# ----------------------------------------------------------- small graphs

def worked_example() -> Graph:
    """The 8-vertex, 8-edge graph of the sweep-cut example (Sec. 3.1).

    A..H = 0..7.  The edges of A, B, C, D follow from the printed Z array;
    the eighth edge (G-H) lies outside {A, B, C, D} and is a free choice
    (the figure is not available); it only fixes 2m = 16.
    """
    edges = [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (3, 5), (3, 6), (6, 7)]
    return from_edges(8, edges, "worked_example")


def complete(k: int) -> Graph:
    return from_edges(k, [(i, j) for i in range(k) for j in range(i + 1, k)], "K%d" % k)


def star(leaves: int) -> Graph:
    return from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)], "star%d" % leaves)


def path(k: int) -> Graph:
    return from_edges(k, [(i, i + 1) for i in range(k - 1)], "path%d" % k)


def cycle(k: int) -> Graph:
    return from_edges(k, [(i, (i + 1) % k) for i in range(k)], "cycle%d" % k)


def barbell(k: int) -> Graph:
    """Two K_k joined by one bridge edge (k-1, k)."""
    e = [(i, j) for i in range(k) for j in range(i + 1, k)]
    e += [(k + i, k + j) for i in range(k) for j in range(i + 1, k)]
    e.append((k - 1, k))
    return from_edges(2 * k, e, "barbell%d" % k)


def torus3d(side: int) -> Graph:
    """side^3 torus: every vertex joined to its two neighbours in each dimension."""
    n = side ** 3
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % side, (idx // side) % side, idx // (side * side)
    e = []
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        j = ((x + dx) % side) + ((y + dy) % side) * side + ((z + dz) % side) * side * side
        e.append(np.stack([idx, j], 1))
    return from_edges(n, np.concatenate(e, 0), "torus%d" % side)


# Offset range of rand_local: with offsets d drawn with probability
# proportional to 1/d on [1, RANDLOCAL_RANGE], five draws per vertex at
# n = 10^7 leave 49.12 M distinct edges, within 0.05 % of the 49,100,524 the
# paper lists for its randLocal input (Sec. 4, table of inputs).
RANDLOCAL_RANGE = 30_000


def rand_local_edges(n: int, k: int = 5, seed: int = 1,
                     span: int = RANDLOCAL_RANGE) -> np.ndarray:
    """The paper's randLocal input (Sec. 4): every vertex v draws k neighbours
    v + d (mod n), the offset d log-uniform on [1, span] (probability about
    proportional to 1/d, so near ids are favoured).  Returns the drawn (v, w)
    pairs; self pairs and duplicates are dropped when the CSR is built."""
    rng = np.random.default_rng(seed)
    u = np.repeat(np.arange(n, dtype=np.int64), k)
    d = np.floor(np.exp(rng.random(n * k) * np.log(span))).astype(np.int64)
    return np.stack([u, (u + d) % n], 1)


def rand_local(n: int, k: int = 5, seed: int = 1, span: int = RANDLOCAL_RANGE) -> Graph:
    """Symmetric CSR of the randLocal input (see rand_local_edges)."""
    return from_edges(n, rand_local_edges(n, k, seed, span), "randlocal%d_k%d_s%d" % (n, k, seed))


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], 1), "er%d_%g_s%d" % (n, p, seed))


# ---------------------------------------------------------------- queries

@dataclass
class QuerySet:
    seeds: np.ndarray   # int32
    alpha: np.ndarray   # float64
    eps: np.ndarray     # float64


def uniform_seeds(g: Graph, count: int, seed: int = 2) -> np.ndarray:
    """Seeds drawn uniformly (with replacement) from vertices of degree >= 1."""
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(g.deg >= 1)
    return cand[rng.integers(0, len(cand), count)].astype(np.int32)


def degree_weighted_seeds(g: Graph, count: int, rng: np.random.Generator) -> np.ndarray:
    """Seeds drawn with probability proportional to degree (source of a random arc)."""
    arcs = rng.integers(0, g.arcs, count)
    return (np.searchsorted(g.off, arcs, side="right") - 1).astype(np.int32)


def batched_queries(g: Graph, count: int, seed: int = 2, eps_lo=1e-7, eps_hi=1e-5,
                    alphas=(0.01, 0.05)) -> QuerySet:
    """Uniform seeds over deg >= 1, eps log-uniform in [eps_lo, eps_hi], alpha from a set."""
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(g.deg >= 1)
    seeds = cand[rng.integers(0, len(cand), count)].astype(np.int32)
    eps = 10.0 ** rng.uniform(np.log10(eps_lo), np.log10(eps_hi), count)
    alpha = np.asarray(alphas, np.float64)[rng.integers(0, len(alphas), count)]
    return QuerySet(seeds, alpha.astype(np.float64), eps.astype(np.float64))
