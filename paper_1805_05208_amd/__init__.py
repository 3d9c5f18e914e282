"""gbgpu: frontier traversal (BFS, integral-weight SSSP) on one MI355X.

Thin ctypes binding over ``libgbgpu.so`` (built from ``csrc/`` by
``_build.py``).  This module only marshals arguments: every step of the
traversal runs in the library's HIP kernels.  PyTorch provides device memory
(tensors) and streams.  There is no CPU fallback -- if the library is missing
the import of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbgpu.so")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP, E_OVERFLOW, E_AGAIN, E_NOTFOUND = range(8)
SYMMETRIC, VALIDATE, SIGNED_WEIGHTS = 1, 2, 4
QUERY_BFS, QUERY_WBFS = 0, 1
BFS_INF = 2**31 - 1
WBFS_INF = 0xFFFFFFFF

EXPORTED = [
    "gbgpu_last_error", "gbgpu_version", "gbgpu_load_csr", "gbgpu_graph_free",
    "gbgpu_graph_info", "gbgpu_bfs", "gbgpu_wbfs", "gbgpu_bellman_ford", "gbgpu_widest_path",
    "gbgpu_bc", "gbgpu_ldd", "gbgpu_connectivity",
    "gbgpu_compress", "gbgpu_decompress", "gbgpu_bfs_compressed", "gbgpu_bfs_simple",
    "gbgpu_bfs_many", "gbgpu_bfs_noalloc",
    "gbgpu_bfs_multi", "gbgpu_bfs_batch",
    "gbgpu_server_create", "gbgpu_server_add_graph", "gbgpu_submit", "gbgpu_poll",
    "gbgpu_server_drain", "gbgpu_server_destroy", "gbgpu_query_footprint",
    "gbgpu_debug_bfs_log", "gbgpu_debug_wbfs_log", "gbgpu_debug_arena_selftest",
    "gbgpu_debug_bfs_join",
]


class GbgpuError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gbgpu status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("force_direction", ctypes.c_int32), ("tau", ctypes.c_int32),
        ("pull_light", ctypes.c_int32), ("wave_chunk", ctypes.c_int32),
        ("grid", ctypes.c_int32), ("bucket_window", ctypes.c_int32),
        ("bucket_capacity", ctypes.c_int32), ("rounds_per_sync", ctypes.c_int32),
        ("profile", ctypes.c_int32), ("max_pending", ctypes.c_int32),
        ("beta", ctypes.c_int32), ("persistent", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32), ("push_rounds", ctypes.c_int32),
        ("pull_rounds", ctypes.c_int32), ("launches", ctypes.c_int32),
        ("reached", ctypes.c_int64), ("edges_examined", ctypes.c_int64),
        ("kernel_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
        ("retries", ctypes.c_int32), ("bucket_peak", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 6),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Query(ctypes.Structure):
    _fields_ = [
        ("graph_id", ctypes.c_int32), ("kind", ctypes.c_int32), ("src", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("dist", ctypes.c_void_p), ("parent", ctypes.c_void_p),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("t_arrive_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64), ("retries", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("join_round", ctypes.c_int32), ("launches", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgbgpu.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, U32, U64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_uint64)
        sig = {
            "gbgpu_last_error": ([], ctypes.c_char_p),
            "gbgpu_version": ([], ctypes.c_int),
            "gbgpu_load_csr": ([I64, I64, P, P, P, U32, P, P], ctypes.c_int),
            "gbgpu_graph_free": ([P], ctypes.c_int),
            "gbgpu_graph_info": ([P, P, P, P], ctypes.c_int),
            "gbgpu_bfs": ([P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_bfs_many": ([P, P, I32, P, P, I64, P, P, P], ctypes.c_int),
            "gbgpu_bfs_noalloc": ([P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_wbfs": ([P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_bellman_ford": ([P, I32, P, P, P, P], ctypes.c_int),
            "gbgpu_widest_path": ([P, I32, P, P, P, P], ctypes.c_int),
            "gbgpu_bc": ([P, I32, P, P, P, P], ctypes.c_int),
            "gbgpu_ldd": ([P, ctypes.c_double, ctypes.c_uint64, P, P, P, P], ctypes.c_int),
            "gbgpu_compress": ([P, P, P], ctypes.c_int),
            "gbgpu_decompress": ([P, P, P], ctypes.c_int),
            "gbgpu_bfs_compressed": ([P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_bfs_simple": ([P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_connectivity": ([P, ctypes.c_double, ctypes.c_uint64, P, P, P, P], ctypes.c_int),
            "gbgpu_bfs_multi": ([P, P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_bfs_batch": ([P, P, I32, P, P, P, P, P], ctypes.c_int),
            "gbgpu_server_create": ([P, ctypes.c_size_t, I32, P, P], ctypes.c_int),
            "gbgpu_server_add_graph": ([P, P, P], ctypes.c_int),
            "gbgpu_submit": ([P, P, P], ctypes.c_int),
            "gbgpu_poll": ([P, U64, P], ctypes.c_int),
            "gbgpu_server_drain": ([P], ctypes.c_int),
            "gbgpu_server_destroy": ([P], ctypes.c_int),
            "gbgpu_query_footprint": ([P, I32, P], ctypes.c_int),
            "gbgpu_debug_bfs_log": ([P, P, I32, P], ctypes.c_int),
            "gbgpu_debug_wbfs_log": ([P, P, I32, P], ctypes.c_int),
            "gbgpu_debug_arena_selftest": ([U64, I32], ctypes.c_int),
            "gbgpu_debug_bfs_join": ([P, P, I32, I32, I32, P, P, P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise GbgpuError(status, lib().gbgpu_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


_OPTS_CACHE: dict = {}


def make_opts(opts) -> Optional[Opts]:
    if opts is None:
        return None
    if isinstance(opts, Opts):
        return opts
    key = tuple(sorted((k, int(v)) for k, v in dict(opts).items()))
    o = _OPTS_CACHE.get(key)
    if o is None:
        o = Opts()
        for k, v in key:
            setattr(o, k, v)
        if len(_OPTS_CACHE) < 256:
            _OPTS_CACHE[key] = o
    return o


def _opts_ref(opts):
    o = make_opts(opts)
    return (ctypes.byref(o) if o is not None else None), o


def _dev_tensor(a, dtype) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dtype).cuda()
    return t.contiguous()


class Graph:
    """A CSR graph resident in device memory plus its library handle.

    The device tensors are owned by this object and kept alive until
    :meth:`free` (the library borrows them)."""

    def __init__(self, offsets, nbrs, weights=None, validate: bool = True, stream=None,
                 name: str = "", signed_weights: bool = False):
        self.offsets = _dev_tensor(offsets, torch.int64)
        self.nbrs = _dev_tensor(nbrs, torch.int32)
        if self.nbrs.numel() == 0:
            self.nbrs = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.weights = None if weights is None else _dev_tensor(weights, torch.int32)
        if self.weights is not None and self.weights.numel() == 0:
            self.weights = torch.ones(1, dtype=torch.int32, device="cuda")
        self.n = int(self.offsets.numel() - 1)
        self.m = int(offsets[-1]) if not isinstance(offsets, torch.Tensor) else int(self.offsets[-1].item())
        self.name = name
        h = ctypes.c_void_p()
        flags = SYMMETRIC | (VALIDATE if validate else 0) | (SIGNED_WEIGHTS if signed_weights else 0)
        _check(lib().gbgpu_load_csr(
            self.n, self.m, ctypes.c_void_p(self.offsets.data_ptr()),
            ctypes.c_void_p(self.nbrs.data_ptr()),
            None if self.weights is None else ctypes.c_void_p(self.weights.data_ptr()),
            flags, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        mw = ctypes.c_int32()
        _check(lib().gbgpu_graph_info(h, None, None, ctypes.byref(mw)))
        self.max_weight = int(mw.value)

    @classmethod
    def from_csr(cls, g, validate: bool = True, with_weights: bool = True, stream=None,
                 signed_weights: bool = False):
        """From a host CSR (graphgen.CSR-like object with offsets/nbrs/weights)."""
        w = g.weights if with_weights else None
        return cls(g.offsets, g.nbrs, w, validate=validate, stream=stream,
                   name=getattr(g, "name", ""), signed_weights=signed_weights)

    def free(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().gbgpu_graph_free(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def bfs_log(self, max_rounds: int = 8192) -> np.ndarray:
        out = np.zeros(max_rounds * 4, dtype=np.uint32)
        nr = ctypes.c_int32()
        _check(lib().gbgpu_debug_bfs_log(self.handle, ctypes.c_void_p(out.ctypes.data),
                                         max_rounds, ctypes.byref(nr)))
        return out[: nr.value * 4].reshape(-1, 4)

    def wbfs_log(self, max_steps: int = 16384) -> np.ndarray:
        out = np.zeros(max_steps * 4, dtype=np.uint32)
        nr = ctypes.c_int32()
        _check(lib().gbgpu_debug_wbfs_log(self.handle, ctypes.c_void_p(out.ctypes.data),
                                          max_steps, ctypes.byref(nr)))
        return out[: nr.value * 4].reshape(-1, 4)

    def footprint(self, kind: int) -> int:
        b = ctypes.c_size_t()
        _check(lib().gbgpu_query_footprint(self.handle, kind, ctypes.byref(b)))
        return int(b.value)


def _out(t, n, dtype):
    if t is None:
        return torch.empty(n, dtype=dtype, device="cuda")
    assert t.is_cuda and t.is_contiguous() and t.numel() >= n
    return t


def bfs(g: Graph, src: int, dist=None, parent=None, opts=None, stream=None,
        stats: bool = False):
    """Single-source BFS.  Returns (dist int32[n], parent int32[n]) device
    tensors, plus a stats dict when stats=True."""
    dist = _out(dist, g.n, torch.int32)
    parent = _out(parent, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bfs(g.handle, int(src), ctypes.c_void_p(dist.data_ptr()),
                           ctypes.c_void_p(parent.data_ptr()), oref, _st_ref(st, stats),
                           _stream_ptr(stream)))
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def bfs_noalloc(g: Graph, src: int, dist, parent, opts=None, stream=None, stats: bool = False):
    """Single-source BFS through the allocation-free entry point (workspace
    in the library's static device array).  dist and parent are
    caller-provided int32[n] device tensors."""
    dist = _out(dist, g.n, torch.int32)
    parent = _out(parent, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bfs_noalloc(g.handle, int(src), ctypes.c_void_p(dist.data_ptr()),
                                   ctypes.c_void_p(parent.data_ptr()), oref, _st_ref(st, stats),
                                   _stream_ptr(stream)))
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def bfs_many(g: Graph, srcs, dist=None, parent=None, row_stride=None, opts=None, stream=None,
             stats: bool = False):
    """k single-source BFS back to back inside the library.  Without outputs
    given, returns (dist, parent) of shape [k, n]; row_stride 0 makes every
    search write the same n entries."""
    src = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    k = int(src.size)
    if row_stride is None:
        row_stride = g.n
    rows = k if row_stride else 1
    need = (rows - 1) * row_stride + g.n if rows > 1 else g.n
    dist = _out(dist, need, torch.int32)
    parent = _out(parent, need, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bfs_many(g.handle, src.ctypes.data_as(ctypes.c_void_p), k,
                                ctypes.c_void_p(dist.data_ptr()), ctypes.c_void_p(parent.data_ptr()),
                                int(row_stride), oref, _st_ref(st, stats), _stream_ptr(stream)))
    if row_stride == g.n and dist.numel() == k * g.n:
        dist, parent = dist.view(k, g.n), parent.view(k, g.n)
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def wbfs(g: Graph, src: int, dist=None, parent=None, opts=None, stream=None,
         stats: bool = False):
    """Integral-weight SSSP.  dist is returned as int32 storage holding the
    uint32 distances (0xFFFFFFFF = unreachable); use ``as_u32`` to view."""
    dist = _out(dist, g.n, torch.int32)
    parent = _out(parent, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_wbfs(g.handle, int(src), ctypes.c_void_p(dist.data_ptr()),
                            ctypes.c_void_p(parent.data_ptr()), oref, _st_ref(st, stats),
                            _stream_ptr(stream)))
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def bellman_ford(g: Graph, src: int, dist=None, opts=None, stream=None, stats: bool = False):
    """General-weight SSSP.  Returns dist int64[n] (INT64_MAX = unreachable,
    INT64_MIN = minus infinity behind a reachable negative cycle)."""
    dist = _out(dist, g.n, torch.int64)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bellman_ford(g.handle, int(src), ctypes.c_void_p(dist.data_ptr()), oref,
                                    _st_ref(st, stats), _stream_ptr(stream)))
    return (dist, st.as_dict()) if stats else dist


def widest_path(g: Graph, src: int, width=None, opts=None, stream=None, stats: bool = False):
    """Widest (bottleneck) path.  Returns int32 storage holding the uint32
    widths (source 0xFFFFFFFF, unreachable 0); use ``as_u32`` to view."""
    width = _out(width, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_widest_path(g.handle, int(src), ctypes.c_void_p(width.data_ptr()), oref,
                                   _st_ref(st, stats), _stream_ptr(stream)))
    return (width, st.as_dict()) if stats else width


def betweenness(g: Graph, src: int, dep=None, opts=None, stream=None, stats: bool = False):
    """Single-source betweenness dependencies, float64[n] (0 for src and
    for unreachable vertices)."""
    dep = _out(dep, g.n, torch.float64)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bc(g.handle, int(src), ctypes.c_void_p(dep.data_ptr()), oref,
                          _st_ref(st, stats), _stream_ptr(stream)))
    return (dep, st.as_dict()) if stats else dep


def ldd(g: Graph, beta: float = 0.2, seed: int = 0, cluster=None, opts=None, stream=None,
        stats: bool = False):
    """Low-diameter decomposition: int32[n] centre id of every vertex's
    cluster (stats: rounds, reached = number of clusters)."""
    cluster = _out(cluster, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_ldd(g.handle, float(beta), int(seed) & (2**64 - 1),
                           ctypes.c_void_p(cluster.data_ptr()), oref, _st_ref(st, stats),
                           _stream_ptr(stream)))
    return (cluster, st.as_dict()) if stats else cluster


def connectivity(g: Graph, beta: float = 0.2, seed: int = 0, label=None, opts=None, stream=None,
                 stats: bool = False):
    """Connected components: int32[n] smallest vertex id of every vertex's
    component (stats: rounds = recursion levels, reached = components)."""
    label = _out(label, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_connectivity(g.handle, float(beta), int(seed) & (2**64 - 1),
                                    ctypes.c_void_p(label.data_ptr()), oref, _st_ref(st, stats),
                                    _stream_ptr(stream)))
    return (label, st.as_dict()) if stats else label


def bfs_multi(g: Graph, srcs: Sequence[int], dist=None, parent=None, opts=None, stream=None,
              stats: bool = False):
    """k BFS problems on one graph solved together.  Returns (dist, parent)
    of shape [k, n]."""
    s = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    k = int(s.size)
    dist = _out(dist, k * g.n, torch.int32).view(k, g.n) if dist is None else dist
    parent = _out(parent, k * g.n, torch.int32).view(k, g.n) if parent is None else parent
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bfs_multi(g.handle, ctypes.c_void_p(s.ctypes.data), k,
                                 ctypes.c_void_p(dist.data_ptr()),
                                 ctypes.c_void_p(parent.data_ptr()), oref, _st_ref(st, stats),
                                 _stream_ptr(stream)))
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def bfs_join(g: Graph, srcs: Sequence[int], k0: int, join_round: int, stream=None):
    """Diagnostic of round-boundary admission: srcs[:k0] start a packed
    group, srcs[k0:] join it at the first round boundary >= join_round.
    Returns (dist, parent) of shape [len(srcs), n]."""
    s = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    k = int(s.size)
    dist = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    parent = torch.empty((k, g.n), dtype=torch.int32, device="cuda")
    _check(lib().gbgpu_debug_bfs_join(g.handle, ctypes.c_void_p(s.ctypes.data), int(k0),
                                      k - int(k0), int(join_round),
                                      ctypes.c_void_p(dist.data_ptr()),
                                      ctypes.c_void_p(parent.data_ptr()), _stream_ptr(stream)))
    return dist, parent


def bfs_batch(graphs: Sequence[Graph], srcs: Sequence[int], dists=None, parents=None,
              opts=None, stream=None, stats: bool = False):
    """Uneven batch of BFS queries over several graphs in one launch.
    Returns lists of per-query (dist, parent) tensors."""
    nq = len(graphs)
    assert len(srcs) == nq
    if dists is None:
        dists = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for gr in graphs]
    if parents is None:
        parents = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for gr in graphs]
    H = (ctypes.c_void_p * nq)(*[gr.handle.value for gr in graphs])
    S = (ctypes.c_int32 * nq)(*[int(x) for x in srcs])
    D = (ctypes.c_void_p * nq)(*[t.data_ptr() for t in dists])
    Pp = (ctypes.c_void_p * nq)(*[t.data_ptr() for t in parents])
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(lib().gbgpu_bfs_batch(H, S, nq, D, Pp, oref, _st_ref(st, stats), _stream_ptr(stream)))
    return (dists, parents, st.as_dict()) if stats else (dists, parents)


def _st_ref(st, wanted: bool):
    """The stats out-parameter, or NULL when the caller does not want stats
    (the library then skips reading its round log back)."""
    return ctypes.byref(st) if wanted else None


def as_u32(t: torch.Tensor) -> np.ndarray:
    """Host uint32 view of an int32 device tensor holding uint32 values."""
    return t.cpu().numpy().view(np.uint32)


class Server:
    """Continuous-batching query server over resident graphs."""

    def __init__(self, arena_bytes: int, max_inflight: int = 8, opts=None):
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self._opts = make_opts(opts)
        h = ctypes.c_void_p()
        _check(lib().gbgpu_server_create(
            ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(max_inflight),
            ctypes.byref(self._opts) if self._opts is not None else None, ctypes.byref(h)))
        self.handle = h
        self.graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        _check(lib().gbgpu_server_add_graph(self.handle, g.handle, ctypes.byref(gid)))
        self.graphs.append(g)
        return int(gid.value)

    def submit(self, graph_id: int, kind: int, src: int, dist: torch.Tensor,
               parent: torch.Tensor) -> int:
        q = Query(graph_id, kind, int(src), 0, dist.data_ptr(), parent.data_ptr())
        t = ctypes.c_uint64()
        _check(lib().gbgpu_submit(self.handle, ctypes.byref(q), ctypes.byref(t)))
        return int(t.value)

    def try_submit(self, graph_id, kind, src, dist, parent):
        """Like submit, but returns None when the pending queue is full."""
        q = Query(graph_id, kind, int(src), 0, dist.data_ptr(), parent.data_ptr())
        t = ctypes.c_uint64()
        st = lib().gbgpu_submit(self.handle, ctypes.byref(q), ctypes.byref(t))
        if st == E_AGAIN:
            return None
        _check(st)
        return int(t.value)

    def poll(self, ticket: int):
        """Returns a result dict once done, else None."""
        r = Result()
        st = lib().gbgpu_poll(self.handle, int(ticket), ctypes.byref(r))
        if st == E_AGAIN:
            return None
        _check(st)
        return {"status": r.status, "rounds": r.rounds, "t_arrive_ns": r.t_arrive_ns,
                "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns, "retries": r.retries,
                "batch": r.batch, "join_round": r.join_round, "launches": r.launches}

    def drain(self):
        _check(lib().gbgpu_server_drain(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().gbgpu_server_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compress(g: Graph, stream=None) -> int:
    """Builds the graph's compressed copy of its lists; returns its size in
    bytes (lists + per-vertex offsets)."""
    b = ctypes.c_int64(0)
    _check(lib().gbgpu_compress(g.handle, ctypes.byref(b), _stream_ptr(stream)))
    return int(b.value)


def decompress(g: Graph, out=None, stream=None):
    """Neighbour array decoded from the compressed copy (int32[m])."""
    out = _out(out, max(g.m, 1), torch.int32)
    _check(lib().gbgpu_decompress(g.handle, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out[: g.m]


def _bfs_lists(fn, g, src, dist, parent, opts, stream, stats):
    dist = _out(dist, g.n, torch.int32)
    parent = _out(parent, g.n, torch.int32)
    oref, _keep = _opts_ref(opts)
    st = Stats()
    _check(fn(g.handle, int(src), ctypes.c_void_p(dist.data_ptr()),
              ctypes.c_void_p(parent.data_ptr()), oref, _st_ref(st, stats), _stream_ptr(stream)))
    return (dist, parent, st.as_dict()) if stats else (dist, parent)


def bfs_compressed(g: Graph, src: int, dist=None, parent=None, opts=None, stream=None,
                   stats: bool = False):
    """BFS reading only the compressed lists (call compress first)."""
    return _bfs_lists(lib().gbgpu_bfs_compressed, g, src, dist, parent, opts, stream, stats)


def bfs_simple(g: Graph, src: int, dist=None, parent=None, opts=None, stream=None,
               stats: bool = False):
    """The same rounds as bfs_compressed over the plain lists."""
    return _bfs_lists(lib().gbgpu_bfs_simple, g, src, dist, parent, opts, stream, stats)
