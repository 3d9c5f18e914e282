"""Pins for the general-weight SSSP (Bellman-Ford) and widest-path oracles
(CPU only).

Each is checked against something other than itself:
  * Bellman-Ford: Floyd-Warshall with minus-infinity propagation on every
    small random directed graph with weights of both signs; scipy's Dijkstra
    and the oracle's own Dial search (a different algorithm) on non-negative
    weights; the closed form of a symmetric graph holding a negative edge
    (every vertex of that edge's component is minus infinity); zero weights.
  * Widest path: the maximum over all simple paths of the smallest weight,
    enumerated on small graphs; the bottleneck on the maximum spanning forest
    (Kruskal's order: the weight at which a vertex joins the source's set);
    closed forms on paths, stars and constant weights.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle

INF64 = int(oracle.SSSP_INF)
NEG64 = int(oracle.SSSP_NEG_INF)
SRC_W = int(oracle.WIDE_SRC)


def _csr_from_edges(n, edges):
    """edges: list of (u, v, w) directed entries; returns a CSR with sorted lists."""
    edges = sorted(edges)
    off = np.zeros(n + 1, dtype=np.int64)
    for u, _, _ in edges:
        off[u + 1] += 1
    g = gg.CSR(n=n, offsets=np.cumsum(off),
               nbrs=np.array([v for _, v, _ in edges], dtype=np.int32))
    g.weights = np.array([w for _, _, w in edges], dtype=np.int32)
    return g


def _symmetric_edges(n, und):
    return [(u, v, w) for u, v, w in und] + [(v, u, w) for u, v, w in und]


# ---------------------------------------------------------------------------
# Bellman-Ford
# ---------------------------------------------------------------------------

def _fw_with_neg_cycles(n, edges, s):
    """Floyd-Warshall over the directed edges, then D[s][v] = -inf when some k
    with D[k][k] < 0 is reachable from s and reaches v."""
    D = np.full((n, n), np.inf)
    for i in range(n):
        D[i, i] = 0.0
    for u, v, w in edges:
        D[u, v] = min(D[u, v], float(w))
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    out = []
    for v in range(n):
        if not np.isfinite(D[s, v]):
            out.append(INF64)
            continue
        neg = any(np.isfinite(D[s, k]) and D[k, k] < 0 and np.isfinite(D[k, v]) for k in range(n))
        out.append(NEG64 if neg else int(D[s, v]))
    return np.array(out, dtype=np.int64)


def test_bellman_ford_brute_force_directed():
    rng = np.random.default_rng(1)
    for _ in range(400):
        n = int(rng.integers(1, 7))
        edges = []
        for u in range(n):
            for v in range(n):
                if u != v and rng.random() < 0.35:
                    edges.append((u, v, int(rng.integers(-3, 6))))
        g = _csr_from_edges(n, edges)
        for s in range(n):
            assert np.array_equal(oracle.bellman_ford(g, s), _fw_with_neg_cycles(n, edges, s)), (n, edges, s)


@pytest.mark.parametrize("scale", [8, 11])
def test_bellman_ford_matches_scipy_and_dial(scale):
    g = gg.rmat(scale, seed=5)
    w = gg.weights(g, 24, seed=6)
    M = sp.csr_matrix((w.astype(np.float64), g.nbrs, g.offsets), shape=(g.n, g.n))
    for s in gg.sources(g, 4, seed=7):
        s = int(s)
        d = oracle.bellman_ford(g, s, w)
        ref = shortest_path(M, method="D", indices=s)
        fin = np.isfinite(ref)
        exp = np.full(g.n, INF64, dtype=np.int64)
        exp[fin] = ref[fin].astype(np.int64)
        assert np.array_equal(d, exp)
        dd, _ = oracle.wbfs(g, s, w)
        exp2 = np.where(dd == oracle.WBFS_INF, INF64, dd.astype(np.int64))
        assert np.array_equal(d, exp2)


def test_bellman_ford_negative_edge_in_symmetric_graph():
    # two components; a negative edge in the source's component makes the
    # whole component minus infinity (u -> v -> u is a negative cycle)
    und = [(0, 1, 4), (1, 2, -1), (2, 3, 2), (4, 5, 3), (5, 6, -2)]
    g = _csr_from_edges(8, _symmetric_edges(8, und))
    d = oracle.bellman_ford(g, 0)
    assert list(d[:4]) == [NEG64] * 4
    assert list(d[4:]) == [INF64] * 4
    # a source in a component without negative edges is unaffected
    und2 = [(0, 1, 4), (1, 2, 1), (4, 5, 3), (5, 6, -2)]
    g2 = _csr_from_edges(8, _symmetric_edges(8, und2))
    assert list(oracle.bellman_ford(g2, 1)) == [4, 0, 1] + [INF64] * 5


def test_bellman_ford_zero_weights_and_unit_reduction():
    und = [(0, 1, 0), (1, 2, 0), (2, 3, 5), (0, 3, 7)]
    g = _csr_from_edges(5, _symmetric_edges(5, und))
    assert list(oracle.bellman_ford(g, 0)) == [0, 0, 0, 5, INF64]
    g = gg.rmat(11, seed=21)
    for s in gg.sources(g, 3, seed=3):
        s = int(s)
        db, _ = oracle.bfs(g, s)
        d = oracle.bellman_ford(g, s, np.ones(g.m, dtype=np.int32))
        exp = np.where(db == oracle.BFS_INF, INF64, db.astype(np.int64))
        assert np.array_equal(d, exp)


def test_bellman_ford_rejects_bad_arguments():
    g = _csr_from_edges(3, _symmetric_edges(3, [(0, 1, 1)]))
    with pytest.raises(ValueError):
        oracle.bellman_ford(g, 3)
    with pytest.raises(ValueError):
        oracle.bellman_ford(g, -1)


# ---------------------------------------------------------------------------
# Widest path
# ---------------------------------------------------------------------------

def _widest_brute(n, und, s):
    adj = {v: [] for v in range(n)}
    for u, v, w in und:
        adj[u].append((v, w))
        adj[v].append((u, w))
    best = [0] * n
    best[s] = SRC_W

    def walk(u, seen, width):
        for v, w in adj[u]:
            if v in seen:
                continue
            c = min(width, w)
            if c > best[v]:
                best[v] = c
            walk(v, seen | {v}, c)

    walk(s, {s}, SRC_W)
    return np.array(best, dtype=np.uint32)


def test_widest_path_brute_force_small():
    rng = np.random.default_rng(2)
    for _ in range(300):
        n = int(rng.integers(1, 8))
        und = [(u, v, int(rng.integers(1, 6)))
               for u, v in itertools.combinations(range(n), 2) if rng.random() < 0.4]
        g = _csr_from_edges(n, _symmetric_edges(n, und))
        for s in range(n):
            assert np.array_equal(oracle.widest_path(g, s), _widest_brute(n, und, s)), (n, und, s)


def _widest_kruskal(g, w, s):
    """Edges in decreasing weight order joined by union-find: a vertex's width
    is the weight of the edge that first puts it in the source's set."""
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(g.offsets))
    keep = rows < g.nbrs
    u_all, v_all, w_all = rows[keep], g.nbrs[keep].astype(np.int64), w[keep]
    order = np.argsort(-w_all, kind="stable")
    parent = list(range(n))
    members = {v: [v] for v in range(n)}
    width = np.zeros(n, dtype=np.uint32)
    width[s] = SRC_W

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for i in order:
        a, b = find(int(u_all[i])), find(int(v_all[i]))
        if a == b:
            continue
        rs = find(s)
        if a == rs or b == rs:
            other = b if a == rs else a
            for x in members[other]:
                width[x] = w_all[i]
        if len(members[a]) < len(members[b]):
            a, b = b, a
        parent[b] = a
        members[a].extend(members.pop(b))
    return width


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(10, seed=31),
    lambda: gg.erdos_renyi(1 << 10, 6, seed=32),
    lambda: gg.torus3d(8),
    lambda: gg.rmat(10, edge_factor=2, seed=33),  # many small components
])
def test_widest_path_matches_maximum_spanning_forest(make):
    g = make()
    w = gg.weights(g, 24, seed=2)
    for s in gg.sources(g, 3, seed=3):
        s = int(s)
        assert np.array_equal(oracle.widest_path(g, s, w), _widest_kruskal(g, w, s))


def test_widest_path_closed_forms():
    # path 0-1-2-3-4 with weights 5, 3, 4, 1: prefix minima from 0, suffix from 4
    und = [(0, 1, 5), (1, 2, 3), (2, 3, 4), (3, 4, 1)]
    g = _csr_from_edges(6, _symmetric_edges(6, und))
    assert list(oracle.widest_path(g, 0)) == [SRC_W, 5, 3, 3, 1, 0]
    assert list(oracle.widest_path(g, 2)) == [3, 3, SRC_W, 4, 1, 0]
    # star: each leaf's width is its edge weight
    und = [(0, k, k) for k in range(1, 6)]
    g = _csr_from_edges(6, _symmetric_edges(6, und))
    assert list(oracle.widest_path(g, 0)) == [SRC_W, 1, 2, 3, 4, 5]
    assert list(oracle.widest_path(g, 3)) == [3, 1, 2, SRC_W, 3, 3]
    # constant weight c: every reachable vertex has width c
    g = gg.rmat(10, edge_factor=2, seed=34)
    db, _ = oracle.bfs(g, 0)
    wd = oracle.widest_path(g, 0, np.full(g.m, 9, dtype=np.int32))
    reach = db != oracle.BFS_INF
    assert wd[0] == SRC_W
    assert np.all(wd[reach & (np.arange(g.n) != 0)] == 9)
    assert np.all(wd[~reach] == 0)


def test_widest_path_rejects_bad_weights():
    g = _csr_from_edges(3, _symmetric_edges(3, [(0, 1, 0)]))
    with pytest.raises(ValueError):
        oracle.widest_path(g, 0)
