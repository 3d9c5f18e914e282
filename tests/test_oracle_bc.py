"""Pins for the single-source betweenness oracle (CPU only).

S[v] = sum over targets t (t != src, t != v) of sigma_st(v) / sigma_st.  The
oracle (Brandes) is checked against:
  * every shortest path enumerated explicitly on small random graphs, with
    exact rational arithmetic;
  * closed forms: a path from an end and from the middle, a star from its
    centre and from a leaf, the complete graph, the antipode of an even cycle;
  * trees, where every target has one shortest path: S[v] = size of v's
    subtree below it;
  * the counting identity sum_v S[v] = sum over reachable t != src of
    (d(src, t) - 1) (each shortest path to t has d - 1 inner vertices) on
    RMAT, Erdos-Renyi and torus inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle


def _csr_und(n, und):
    edges = sorted(set([(u, v) for u, v in und] + [(v, u) for u, v in und]))
    off = np.zeros(n + 1, dtype=np.int64)
    for u, _ in edges:
        off[u + 1] += 1
    return gg.CSR(n=n, offsets=np.cumsum(off), nbrs=np.array([v for _, v in edges], dtype=np.int32))


def _brute(n, und, s):
    adj = {v: set() for v in range(n)}
    for u, v in und:
        adj[u].add(v)
        adj[v].add(u)
    # all shortest paths from s, enumerated: BFS distances, then every
    # walk that steps one level deeper at each edge
    dist = {s: 0}
    frontier = [s]
    while frontier:
        nxt = []
        for u in frontier:
            for v in adj[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    nxt.append(v)
        frontier = nxt
    paths = {s: [[s]]}
    for v in sorted(dist, key=lambda x: dist[x]):
        if v == s:
            continue
        paths[v] = [p + [v] for u in adj[v] if dist.get(u, -2) == dist[v] - 1 for p in paths[u]]
    S = [Fraction(0)] * n
    for t, ps in paths.items():
        if t == s:
            continue
        for v in range(n):
            if v in (s, t):
                continue
            through = sum(1 for p in ps if v in p)
            S[v] += Fraction(through, len(ps))
    return S


def test_enumerated_shortest_paths_small_graphs():
    rng = np.random.default_rng(3)
    for _ in range(250):
        n = int(rng.integers(1, 8))
        und = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.45]
        g = _csr_und(n, und)
        for s in range(n):
            got = oracle.betweenness(g, s)
            exp = _brute(n, und, s)
            assert np.allclose(got, [float(x) for x in exp], rtol=1e-12, atol=1e-12), (n, und, s)


def test_closed_forms():
    n = 9
    path = _csr_und(n, [(i, i + 1) for i in range(n - 1)])
    assert np.allclose(oracle.betweenness(path, 0), [0] + [n - 1 - v for v in range(1, n)])
    mid = oracle.betweenness(path, 4)
    exp = [0.0] * n
    for v in range(n):
        if v < 4:
            exp[v] = v          # the vertices 0..v-1 lie beyond v
        elif v > 4:
            exp[v] = n - 1 - v
    assert np.allclose(mid, exp)
    star = _csr_und(7, [(0, k) for k in range(1, 7)])
    assert np.allclose(oracle.betweenness(star, 0), 0.0)
    leaf = oracle.betweenness(star, 3)
    assert leaf[0] == 5 and np.allclose(np.delete(leaf, 0), 0.0)
    k6 = _csr_und(6, [(u, v) for u in range(6) for v in range(u + 1, 6)])
    assert np.allclose(oracle.betweenness(k6, 2), 0.0)
    # even cycle C8 from 0: the antipode 4 has two shortest paths; every
    # other target one
    c8 = _csr_und(8, [(i, (i + 1) % 8) for i in range(8)])
    b = oracle.betweenness(c8, 0)
    assert np.allclose(b, [0, 2.5, 1.5, 0.5, 0, 0.5, 1.5, 2.5])


def test_trees_subtree_sizes():
    rng = np.random.default_rng(4)
    for _ in range(50):
        n = int(rng.integers(2, 60))
        par = [-1] + [int(rng.integers(0, v)) for v in range(1, n)]
        g = _csr_und(n, [(v, par[v]) for v in range(1, n)])
        size = [1] * n
        for v in range(n - 1, 0, -1):
            size[par[v]] += size[v]
        exp = [0.0] + [size[v] - 1.0 for v in range(1, n)]
        assert np.allclose(oracle.betweenness(g, 0), exp)


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(13, seed=41),
    lambda: gg.erdos_renyi(1 << 12, 6, seed=42),
    lambda: gg.torus3d(12),
    lambda: gg.rmat(12, edge_factor=2, seed=43),
])
def test_sum_identity(make):
    g = make()
    for s in [int(x) for x in gg.sources(g, 3, seed=3)]:
        dep = oracle.betweenness(g, s)
        d, _ = oracle.bfs(g, s)
        reach = (d != oracle.BFS_INF) & (np.arange(g.n) != s)
        assert dep[s] == 0 and np.all(dep[d == oracle.BFS_INF] == 0)
        assert np.isclose(dep.sum(), float((d[reach].astype(np.int64) - 1).sum()), rtol=1e-10)


def test_rejects_bad_arguments():
    g = _csr_und(3, [(0, 1)])
    with pytest.raises(ValueError):
        oracle.betweenness(g, 3)
