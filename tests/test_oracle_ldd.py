"""Pins for the low-diameter decomposition and connectivity oracles (CPU).

LDD is an iteration, so the oracle runs the paper's rounds; it is pinned to
the definition those rounds reach.  With T(v) = min over all c of
(start(c) + d(c, v)) (the round at which v enters the frontier, computed
here with scipy's Dijkstra from a super-source joined to every c at weight
start(c) + 1), a vertex is a centre iff start(v) <= T(u) for every
neighbour u (nobody could claim it before its own start), and any other
vertex belongs to the cluster of its smallest-ID neighbour u with
T(u) = T(v) - 1.  Also pinned: the shift generator's geometric law, closed
forms (no edges; the complete graph), and connected components against
scipy.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import graphgen as gg
import oracle


def expected_ldd(g, beta, seed, level=0):
    n = g.n
    gs = oracle.geo_shifts(n, beta, seed, level)
    start = gs.max() - gs
    rows = np.repeat(np.arange(n), np.diff(g.offsets))
    # super-source n: edge to every vertex at weight start + 1, graph edges 1
    r = np.concatenate([rows, np.full(n, n)])
    c = np.concatenate([g.nbrs, np.arange(n)])
    w = np.concatenate([np.ones(g.m), start + 1.0])
    M = sp.csr_matrix((w, (r, c)), shape=(n + 1, n + 1))
    T = (shortest_path(M, method="D", indices=n)[:n] - 1).astype(np.int64)
    cl = np.full(n, -1, dtype=np.int64)
    for v in np.argsort(T, kind="stable"):
        nb = g.nbrs[g.offsets[v]:g.offsets[v + 1]]
        if nb.size == 0 or start[v] <= T[nb].min():
            cl[v] = v
        else:
            cand = nb[T[nb] == T[v] - 1]
            cl[v] = cl[cand.min()]
    return cl


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(10, seed=1),
    lambda: gg.rmat(11, edge_factor=4, seed=2),
    lambda: gg.erdos_renyi(1 << 10, 4, seed=3),
    lambda: gg.torus3d(8),
])
@pytest.mark.parametrize("beta", [0.05, 0.2, 0.8])
def test_ldd_matches_definition(make, beta):
    g = make()
    for seed in (1, 99):
        assert np.array_equal(oracle.ldd(g, beta, seed), expected_ldd(g, beta, seed))


def test_ldd_levels_draw_fresh_shifts():
    g = gg.torus3d(6)
    a, b = oracle.ldd(g, 0.3, 5, level=0), oracle.ldd(g, 0.3, 5, level=1)
    assert np.array_equal(b, expected_ldd(g, 0.3, 5, level=1))
    assert not np.array_equal(oracle.geo_shifts(g.n, 0.3, 5, 0), oracle.geo_shifts(g.n, 0.3, 5, 1))
    assert a.shape == b.shape


def test_geometric_shift_law():
    for beta in (0.1, 0.5):
        q = np.exp(-beta)
        x = oracle.geo_shifts(200_000, beta, 12345)
        assert abs(x.mean() - q / (1 - q)) < 0.02 * q / (1 - q)
        for k in (1, 3, 8):
            assert abs((x >= k).mean() - q ** k) < 0.01
        assert x.max() <= 63 and x.min() >= 0


def test_ldd_closed_forms():
    n = 12
    empty = gg.CSR(n=n, offsets=np.zeros(n + 1, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    assert np.array_equal(oracle.ldd(empty, 0.2, 3), np.arange(n))
    rows = [(u, v) for u in range(n) for v in range(n) if u != v]
    off = np.zeros(n + 1, dtype=np.int64)
    for u, _ in rows:
        off[u + 1] += 1
    kn = gg.CSR(n=n, offsets=np.cumsum(off), nbrs=np.array([v for _, v in rows], dtype=np.int32))
    gs = oracle.geo_shifts(n, 0.2, 3)
    centres = np.nonzero(gs == gs.max())[0]
    exp = np.full(n, centres.min())
    exp[centres] = centres
    assert np.array_equal(oracle.ldd(kn, 0.2, 3), exp)


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(12, edge_factor=2, seed=4),
    lambda: gg.erdos_renyi(1 << 12, 1, seed=5),
    lambda: gg.torus3d(10),
    lambda: gg.rmat(10, seed=6),
])
def test_components_match_scipy(make):
    g = make()
    lab = oracle.components(g)
    M = sp.csr_matrix((np.ones(g.m), g.nbrs, g.offsets), shape=(g.n, g.n))
    k, ref = connected_components(M, directed=False)
    # canonical form of scipy's labels: the smallest vertex of each component
    first = np.full(k, g.n)
    np.minimum.at(first, ref, np.arange(g.n))
    assert np.array_equal(lab, first[ref])
