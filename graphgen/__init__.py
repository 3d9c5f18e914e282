"""Seeded synthetic graph inputs shared by the oracle and the GPU path.

Holds input generation only (random draws, CSR assembly, weights, source
picking); no traversal arithmetic.  Every graph is a symmetric CSR:
``offsets`` int64[n+1], ``nbrs`` int32[m] sorted strictly ascending per
vertex, no self loops, no duplicate edges.  Weighted inputs carry ``weights``
int32[m], symmetric per undirected edge, uniform in [1, W).

The large generators (RMAT, Erdos-Renyi, torus, weights) run in C with OpenMP
(``graphgen.c``); small textbook graphs used as test fixtures are built here
with numpy.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        U64 = ctypes.c_uint64
        I = ctypes.c_int
        D = ctypes.c_double
        lib.gg_rmat_edges.argtypes = [I, I64, D, D, D, U64, P, P, I]
        lib.gg_er_edges.argtypes = [I64, I64, U64, P, P, I]
        lib.gg_csr_count.argtypes = [I64, I64, P, P, P, I]
        lib.gg_csr_count.restype = I64
        lib.gg_csr_fill.argtypes = [I64, I64, P, P, P, P, P, P, I]
        lib.gg_csr_fill.restype = I64
        lib.gg_csr_compact.argtypes = [I64, P, P, P, P, P, I]
        lib.gg_torus_degree.argtypes = [I64]
        lib.gg_torus_degree.restype = I64
        lib.gg_torus3d.argtypes = [I64, P, P, I]
        lib.gg_weights.argtypes = [I64, P, P, I64, U64, P, I]
        lib.gg_sources.argtypes = [I64, P, I64, U64, P]
        lib.gg_sources.restype = I64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _threads() -> int:
    env = os.environ.get("GG_THREADS")
    if env:
        return int(env)
    return min(16, os.cpu_count() or 1)


@dataclasses.dataclass
class CSR:
    """Symmetric CSR graph held in host memory."""

    n: int
    offsets: np.ndarray  # int64[n+1]
    nbrs: np.ndarray  # int32[m]
    weights: Optional[np.ndarray] = None  # int32[m] or None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.offsets[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def with_weights(self, W: int, seed: int = 2) -> "CSR":
        return dataclasses.replace(self, weights=weights(self, W, seed),
                                   name=self.name + f"-w{W}")


def _csr_from_raw(n: int, us: np.ndarray, vs: np.ndarray, name: str) -> CSR:
    lib = _load()
    t = _threads()
    ne = int(us.shape[0])
    deg_raw = np.empty(n, dtype=np.int64)
    tot = lib.gg_csr_count(n, ne, _ptr(us), _ptr(vs), _ptr(deg_raw), t)
    tmp = np.empty(max(tot, 1), dtype=np.uint32)
    raw_off = np.empty(n + 1, dtype=np.int64)
    deg = np.empty(n, dtype=np.int64)
    m = lib.gg_csr_fill(n, ne, _ptr(us), _ptr(vs), _ptr(deg_raw), _ptr(tmp),
                        _ptr(raw_off), _ptr(deg), t)
    del deg_raw
    offsets = np.empty(n + 1, dtype=np.int64)
    nbrs = np.empty(max(m, 1), dtype=np.int32)
    lib.gg_csr_compact(n, _ptr(tmp), _ptr(raw_off), _ptr(deg), _ptr(offsets), _ptr(nbrs), t)
    return CSR(n=n, offsets=offsets, nbrs=nbrs[:m], name=name)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1) -> CSR:
    """RMAT graph with 2^scale vertices and edge_factor * 2^scale raw edges,
    symmetrised, without self loops or duplicates."""
    if not (1 <= scale <= 30):
        raise ValueError("scale must be in [1, 30]")
    n = 1 << scale
    ne = edge_factor * n
    us = np.empty(ne, dtype=np.uint32)
    vs = np.empty(ne, dtype=np.uint32)
    _load().gg_rmat_edges(scale, ne, a, b, c, seed, _ptr(us), _ptr(vs), _threads())
    return _csr_from_raw(n, us, vs, f"rmat{scale}-ef{edge_factor}-s{seed}")


def erdos_renyi(n: int, avg_degree: int, seed: int = 1) -> CSR:
    """Erdos-Renyi style graph: n*avg_degree/2 uniform vertex pairs,
    symmetrised, without self loops or duplicates."""
    npairs = n * avg_degree // 2
    us = np.empty(npairs, dtype=np.uint32)
    vs = np.empty(npairs, dtype=np.uint32)
    _load().gg_er_edges(n, npairs, seed, _ptr(us), _ptr(vs), _threads())
    return _csr_from_raw(n, us, vs, f"er{n}-d{avg_degree}-s{seed}")


def torus3d(k: int) -> CSR:
    """k x k x k torus, vertex id x + k*y + k*k*z."""
    lib = _load()
    n = k * k * k
    d = lib.gg_torus_degree(k)
    offsets = np.empty(n + 1, dtype=np.int64)
    nbrs = np.empty(max(n * d, 1), dtype=np.int32)
    lib.gg_torus3d(k, _ptr(offsets), _ptr(nbrs), _threads())
    return CSR(n=n, offsets=offsets, nbrs=nbrs[: n * d], name=f"torus{k}")


def weights(g: CSR, W: int, seed: int = 2) -> np.ndarray:
    """Symmetric integral weights uniform in [1, W) (W >= 2)."""
    if W < 2:
        raise ValueError("W must be >= 2")
    w = np.empty(max(g.m, 1), dtype=np.int32)
    _load().gg_weights(g.n, _ptr(g.offsets), _ptr(g.nbrs), W, seed, _ptr(w), _threads())
    return w[: g.m]


def log2_weight_bound(n: int) -> int:
    """Exclusive weight bound log2(n) used for [1, log2 n) weights."""
    return max(2, int(math.log2(n)))


def sources(g: CSR, k: int, seed: int = 3) -> np.ndarray:
    """k distinct seeded vertices of nonzero degree."""
    out = np.empty(max(k, 1), dtype=np.int32)
    got = _load().gg_sources(g.n, _ptr(g.offsets), k, seed, _ptr(out))
    return out[:got]


# ---------------------------------------------------------------------------
# Small textbook graphs (test fixtures), built with numpy.
# ---------------------------------------------------------------------------

def from_edges(n: int, edges, weights_=None, name: str = "") -> CSR:
    """Symmetric CSR from undirected (u, v) pairs; self loops dropped,
    duplicates merged (the first weight given for a pair is kept)."""
    adj = [dict() for _ in range(n)]
    for i, (u, v) in enumerate(edges):
        u = int(u)
        v = int(v)
        if u == v:
            continue
        w = 1 if weights_ is None else int(weights_[i])
        if v not in adj[u]:
            adj[u][v] = w
            adj[v][u] = w
    offsets = np.zeros(n + 1, dtype=np.int64)
    nb, ww = [], []
    for u in range(n):
        keys = sorted(adj[u])
        nb.extend(keys)
        ww.extend(adj[u][k] for k in keys)
        offsets[u + 1] = offsets[u] + len(keys)
    g = CSR(n=n, offsets=offsets, nbrs=np.array(nb, dtype=np.int32), name=name)
    if weights_ is not None:
        g.weights = np.array(ww, dtype=np.int32)
    return g


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], name=f"path{n}")


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"cycle{n}")


def star(n: int) -> CSR:
    return from_edges(n, [(0, i) for i in range(1, n)], name=f"star{n}")


def complete(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)],
                      name=f"complete{n}")


def grid2d(a: int, b: int) -> CSR:
    """a x b grid (no wrap), vertex id x + a*y."""
    e = []
    for y in range(b):
        for x in range(a):
            v = x + a * y
            if x + 1 < a:
                e.append((v, v + 1))
            if y + 1 < b:
                e.append((v, v + a))
    return from_edges(a * b, e, name=f"grid{a}x{b}")


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """Graph with vertex v renamed perm[v] (lists re-sorted)."""
    n = g.n
    deg = g.degrees()
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    nu = perm[src].astype(np.int64)
    nv = perm[g.nbrs.astype(np.int64)].astype(np.int64)
    order = np.lexsort((nv, nu))
    nu, nv = nu[order], nv[order]
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offsets, nu + 1, 1)
    offsets = np.cumsum(offsets)
    out = CSR(n=n, offsets=offsets, nbrs=nv.astype(np.int32), name=g.name + "-perm")
    if g.weights is not None:
        out.weights = g.weights[order].astype(np.int32)
    return out
