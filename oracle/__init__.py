"""Oracle for BFS and integral-weight SSSP -- TEST INFRASTRUCTURE ONLY.

Plain sequential CPU code (``oracle.c``) that defines the expected outputs of
the GPU library.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU path: the only common dependency is the seeded input generator
package ``graphgen``, which holds no traversal arithmetic.

Functions follow the problem statements of the Benchmark section ("Shortest
Path Problems"), with parents fixed by the minimum-ID rule:

* :func:`bfs`  -- hop distances (int32, INT32_MAX = unreachable) and
  parent[v] = min{u in N(v): D[u] + 1 == D[v]}, parent[src] = src, -1 if
  unreachable.
* :func:`wbfs` -- integral-weight distances (uint32, 0xFFFFFFFF =
  unreachable), computed with Dial's bucketed Dijkstra, and
  parent[v] = min{u in N(v): D[u] + w(u,v) == D[v]}.
* :func:`bellman_ford` -- general-weight SSSP distances (int64, INT64_MAX =
  unreachable, INT64_MIN = minus infinity behind a reachable negative
  cycle), textbook Bellman-Ford.
* :func:`widest_path` -- widest (bottleneck) path widths (uint32, source =
  0xFFFFFFFF, unreachable = 0), Dijkstra on a max-heap of widths.
* :func:`betweenness` -- single-source betweenness dependencies (float64,
  0 for the source and unreachable vertices), textbook Brandes.
* :func:`ldd` -- low-diameter decomposition clusters (int32 centre ids),
  the paper's LDD rounds with geometric shifts from SplitMix64 and the
  smallest-ID-claimer rule; :func:`geo_shifts` returns the shifts.
* :func:`components` -- connected components, labelled by their smallest
  vertex id.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

BFS_INF = np.int32(2**31 - 1)
WBFS_INF = np.uint32(0xFFFFFFFF)
SSSP_INF = np.int64(2**63 - 1)
SSSP_NEG_INF = np.int64(-2**63)
WIDE_SRC = np.uint32(0xFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile oracle.c (plain C, -O3, single-threaded) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_bfs.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P]
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_wbfs.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, P]
        lib.oracle_wbfs.restype = ctypes.c_int
        lib.oracle_bellman_ford.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P]
        lib.oracle_bellman_ford.restype = ctypes.c_int
        lib.oracle_widest_path.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P]
        lib.oracle_widest_path.restype = ctypes.c_int
        lib.oracle_betweenness.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P]
        lib.oracle_betweenness.restype = ctypes.c_int
        lib.oracle_geo_threshold.argtypes = [ctypes.c_double]
        lib.oracle_geo_threshold.restype = ctypes.c_uint64
        lib.oracle_geo_shift.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint64]
        lib.oracle_geo_shift.restype = ctypes.c_int32
        lib.oracle_ldd.argtypes = [ctypes.c_int64, P, P, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_uint32, P]
        lib.oracle_ldd.restype = ctypes.c_int
        lib.oracle_components.argtypes = [ctypes.c_int64, P, P, P]
        lib.oracle_components.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _csr_arrays(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    nb = np.ascontiguousarray(g.nbrs, dtype=np.int32)
    if nb.size == 0:
        nb = np.zeros(1, dtype=np.int32)
    return off, nb


def bfs(g, src: int):
    """Return (dist int32[n], parent int32[n]) for a BFS from src."""
    off, nb = _csr_arrays(g)
    dist = np.empty(g.n, dtype=np.int32)
    parent = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_bfs(g.n, _p(off), _p(nb), int(src), _p(dist), _p(parent))
    if rc != 0:
        raise ValueError(f"oracle_bfs failed with code {rc}")
    return dist, parent


def wbfs(g, src: int, weights=None):
    """Return (dist uint32[n], parent int32[n]) for integral-weight SSSP."""
    w = g.weights if weights is None else weights
    if w is None:
        raise ValueError("weighted graph required")
    off, nb = _csr_arrays(g)
    ww = np.ascontiguousarray(w, dtype=np.int32)
    if ww.size == 0:
        ww = np.ones(1, dtype=np.int32)
    dist = np.empty(g.n, dtype=np.uint32)
    parent = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_wbfs(g.n, _p(off), _p(nb), _p(ww), int(src), _p(dist), _p(parent))
    if rc != 0:
        raise ValueError(f"oracle_wbfs failed with code {rc}")
    return dist, parent


def _weights_of(g, weights):
    w = g.weights if weights is None else weights
    if w is None:
        raise ValueError("weighted graph required")
    ww = np.ascontiguousarray(w, dtype=np.int32)
    if ww.size == 0:
        ww = np.ones(1, dtype=np.int32)
    return ww


def bellman_ford(g, src: int, weights=None):
    """Return dist int64[n] for general-weight SSSP (any int32 weights)."""
    off, nb = _csr_arrays(g)
    ww = _weights_of(g, weights)
    dist = np.empty(g.n, dtype=np.int64)
    rc = _load().oracle_bellman_ford(g.n, _p(off), _p(nb), _p(ww), int(src), _p(dist))
    if rc != 0:
        raise ValueError(f"oracle_bellman_ford failed with code {rc}")
    return dist


def widest_path(g, src: int, weights=None):
    """Return width uint32[n] for the widest (bottleneck) path problem."""
    off, nb = _csr_arrays(g)
    ww = _weights_of(g, weights)
    width = np.empty(g.n, dtype=np.uint32)
    rc = _load().oracle_widest_path(g.n, _p(off), _p(nb), _p(ww), int(src), _p(width))
    if rc != 0:
        raise ValueError(f"oracle_widest_path failed with code {rc}")
    return width


def betweenness(g, src: int):
    """Return dep float64[n]: S[v] = sum over targets t of sigma_st(v) / sigma_st."""
    off, nb = _csr_arrays(g)
    dep = np.empty(g.n, dtype=np.float64)
    rc = _load().oracle_betweenness(g.n, _p(off), _p(nb), int(src), _p(dep))
    if rc != 0:
        raise ValueError(f"oracle_betweenness failed with code {rc}")
    return dep


def geo_shifts(n: int, beta: float, seed: int, level: int = 0) -> np.ndarray:
    """The LDD shifts g(v) (int32[n])."""
    L = _load()
    thr = L.oracle_geo_threshold(float(beta))
    return np.array([L.oracle_geo_shift(seed, level, v, thr) for v in range(n)], dtype=np.int32)


def ldd(g, beta: float, seed: int, level: int = 0):
    """Return cluster int32[n] (centre id of every vertex's cluster)."""
    off, nb = _csr_arrays(g)
    cl = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_ldd(g.n, _p(off), _p(nb), float(beta), int(seed) & (2**64 - 1),
                            int(level), _p(cl))
    if rc != 0:
        raise ValueError(f"oracle_ldd failed with code {rc}")
    return cl


def components(g):
    """Return label int32[n] = smallest vertex id of each vertex's component."""
    off, nb = _csr_arrays(g)
    lab = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_components(g.n, _p(off), _p(nb), _p(lab))
    if rc != 0:
        raise ValueError(f"oracle_components failed with code {rc}")
    return lab
