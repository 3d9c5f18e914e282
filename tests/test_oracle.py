"""Pins for the oracle (CPU only).

The oracle is checked against things other than itself:
  * hand-worked fixtures in tests/golden (problem statements of the Benchmark
    section, "Shortest Path Problems");
  * brute force on every undirected graph with up to 6 vertices (Floyd-Warshall
    distances, parents enumerated from the min-ID definition);
  * closed forms: path, cycle (even cycles give the antipodal parent tie),
    star, complete graph, 2-D grid, 3-D torus (the paper's high-diameter
    family, Experiments, "Graph Data");
  * a library routine (scipy's Dijkstra / unweighted shortest paths);
  * definition-level invariants (tests/checks.py) on RMAT, Erdos-Renyi and
    torus inputs;
  * reductions: unit weights give wBFS == BFS; constant weight c scales BFS.
A mutation test shows the checks reject plausible slips (a dropped parent
minimum, an off-by-one level, a wrong weight term).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle
from checks import BFS_INF, WBFS_INF, check_bfs, check_wbfs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _parse_golden(name):
    rows = {}
    edges = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, *vals = line.split()
            if k == "edge":
                edges.append(tuple(int(x) for x in vals))
            else:
                rows[k] = vals
    n = int(rows["n"][0])
    src = int(rows["src"][0])
    g = gg.from_edges(n, [(u, v) for u, v, _ in edges], [w for _, _, w in edges])
    return g, src, rows


def _vals(tokens, inf):
    return np.array([inf if t == "inf" else int(t) for t in tokens], dtype=np.int64)


@pytest.mark.parametrize("name", ["small_unweighted.txt", "small_weighted.txt"])
def test_golden_fixtures(name):
    g, src, rows = _parse_golden(name)
    d, p = oracle.bfs(g, src)
    assert np.array_equal(d.astype(np.int64), _vals(rows["bfs_dist"], BFS_INF))
    assert np.array_equal(p.astype(np.int64), _vals(rows["bfs_parent"], -1))
    check_bfs(g, src, d, p)
    if "wbfs_dist" in rows:
        d, p = oracle.wbfs(g, src)
        assert np.array_equal(d.astype(np.int64), _vals(rows["wbfs_dist"], WBFS_INF))
        assert np.array_equal(p.astype(np.int64), _vals(rows["wbfs_parent"], -1))
        check_wbfs(g, src, d, p)


# ---------------------------------------------------------------------------
# Exhaustive brute force on tiny graphs
# ---------------------------------------------------------------------------

def _all_graphs(n):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    G = 1 << len(pairs)
    A = np.zeros((G, n, n), dtype=bool)
    masks = np.arange(G)
    for b, (i, j) in enumerate(pairs):
        bit = ((masks >> b) & 1).astype(bool)
        A[:, i, j] = bit
        A[:, j, i] = bit
    return A


def _floyd_warshall(W):
    """W[G, n, n] edge weights (inf for none); returns all-pairs distances."""
    n = W.shape[-1]
    D = W.copy()
    idx = np.arange(n)
    D[:, idx, idx] = 0
    for k in range(n):
        D = np.minimum(D, D[:, :, k:k + 1] + D[:, k:k + 1, :])
    return D


def _def_parents(A, W, D):
    """parent[G, s, v] = min{u : A[v,u], D[s,u] + W[u,v] == D[s,v]}, s for v == s,
    -1 if unreachable -- the definition, enumerated."""
    G, n, _ = A.shape
    cand = (A[:, None, :, :]
            & np.isfinite(D)[:, :, None, :]
            & (D[:, :, None, :] + W[:, None, :, :] == D[:, :, :, None]))
    u_idx = np.where(cand, np.arange(n)[None, None, None, :], n)
    par = u_idx.min(axis=-1)
    par = np.where(par == n, -1, par)
    s = np.arange(n)
    par[:, s, s] = s
    par = np.where(np.isfinite(D), par, -1)
    return par


def _csr_of(Arow, Wrow=None):
    n = Arow.shape[0]
    rows, cols = np.nonzero(Arow)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offsets, rows + 1, 1)
    g = gg.CSR(n=n, offsets=np.cumsum(offsets), nbrs=cols.astype(np.int32))
    if Wrow is not None:
        g.weights = Wrow[rows, cols].astype(np.int32)
    return g


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_bfs_exhaustive_tiny_graphs(n):
    A = _all_graphs(n)
    W = np.where(A, 1.0, np.inf)
    D = _floyd_warshall(W)
    P = _def_parents(A, W, D)
    Dint = np.where(np.isfinite(D), D, BFS_INF).astype(np.int64)
    for gi in range(A.shape[0]):
        g = _csr_of(A[gi])
        for s in range(n):
            d, p = oracle.bfs(g, s)
            if not (np.array_equal(d, Dint[gi, s]) and np.array_equal(p, P[gi, s])):
                raise AssertionError(f"graph {gi} src {s}: {d} {p} vs {Dint[gi, s]} {P[gi, s]}")


@pytest.mark.parametrize("n", [3, 4, 5])
def test_wbfs_exhaustive_tiny_graphs(n):
    A = _all_graphs(n)
    rng = np.random.default_rng(100 + n)
    w = rng.integers(1, 5, size=A.shape)
    w = np.triu(w, 1)
    w = w + np.transpose(w, (0, 2, 1))
    W = np.where(A, w.astype(float), np.inf)
    D = _floyd_warshall(W)
    P = _def_parents(A, W, D)
    Dint = np.where(np.isfinite(D), D, WBFS_INF).astype(np.int64)
    for gi in range(A.shape[0]):
        g = _csr_of(A[gi], w[gi])
        for s in range(n):
            d, p = oracle.wbfs(g, s)
            assert np.array_equal(d.astype(np.int64), Dint[gi, s]), (gi, s)
            assert np.array_equal(p, P[gi, s]), (gi, s)


def test_random_small_graphs_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(2, 13))
        p = rng.uniform(0.1, 0.6)
        A = rng.random((n, n)) < p
        A = np.triu(A, 1)
        A = A | A.T
        w = np.triu(rng.integers(1, 9, size=(n, n)), 1)
        w = w + w.T
        Wu = np.where(A, 1.0, np.inf)[None]
        Ww = np.where(A, w.astype(float), np.inf)[None]
        Du = _floyd_warshall(Wu)
        Dw = _floyd_warshall(Ww)
        Pu = _def_parents(A[None], Wu, Du)[0]
        Pw = _def_parents(A[None], Ww, Dw)[0]
        g = _csr_of(A, w)
        for s in range(n):
            d, pp = oracle.bfs(g, s)
            assert np.array_equal(d, np.where(np.isfinite(Du[0, s]), Du[0, s], BFS_INF).astype(np.int64))
            assert np.array_equal(pp, Pu[s])
            d, pp = oracle.wbfs(g, s)
            assert np.array_equal(d.astype(np.int64),
                                  np.where(np.isfinite(Dw[0, s]), Dw[0, s], WBFS_INF).astype(np.int64))
            assert np.array_equal(pp, Pw[s])


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def test_path_closed_form():
    for n in range(1, 20):
        g = gg.path(n)
        for s in range(n):
            d, p = oracle.bfs(g, s)
            v = np.arange(n)
            assert np.array_equal(d, np.abs(v - s))
            exp = np.where(v < s, v + 1, v - 1)
            exp[s] = s
            assert np.array_equal(p, exp)


def test_cycle_closed_form_and_antipode_tie():
    for n in range(3, 24):
        g = gg.cycle(n)
        for s in range(n):
            d, p = oracle.bfs(g, s)
            v = np.arange(n)
            delta = np.abs(v - s)
            assert np.array_equal(d, np.minimum(delta, n - delta))
            # parent: neighbours one step closer; the antipode of an even
            # cycle has two and takes the smaller id
            for x in range(n):
                if x == s:
                    assert p[x] == s
                    continue
                nb = [(x - 1) % n, (x + 1) % n]
                closer = [y for y in nb if d[y] == d[x] - 1]
                assert p[x] == min(closer)
            if n % 2 == 0:
                a = (s + n // 2) % n
                assert p[a] == min((a - 1) % n, (a + 1) % n)


def test_star_and_complete():
    for n in (2, 5, 17):
        g = gg.star(n)
        d, p = oracle.bfs(g, 0)
        assert np.all(d[1:] == 1) and np.all(p[1:] == 0)
        d, p = oracle.bfs(g, n - 1)
        if n > 2:
            assert d[0] == 1 and np.all(d[1:n - 1] == 2) and np.all(p[1:n - 1] == 0)
        g = gg.complete(n)
        for s in range(n):
            d, p = oracle.bfs(g, s)
            exp = np.full(n, s)
            assert np.all(d[np.arange(n) != s] == 1) and np.array_equal(p, exp)


def test_grid_manhattan():
    rng = np.random.default_rng(3)
    for _ in range(10):
        a, b = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        g = gg.grid2d(a, b)
        s = int(rng.integers(0, a * b))
        d, p = oracle.bfs(g, s)
        x, y = np.arange(a * b) % a, np.arange(a * b) // a
        sx, sy = s % a, s // a
        assert np.array_equal(d, np.abs(x - sx) + np.abs(y - sy))
        check_bfs(g, s, d, p)


def torus_closed_form(k, s):
    """BFS distances and min-ID parents on the k^3 torus, from the closed
    form d = sum over dimensions of min(|delta|, k - |delta|)."""
    n = k ** 3
    v = np.arange(n, dtype=np.int64)
    co = np.stack([v % k, (v // k) % k, v // (k * k)])
    sc = np.array([s % k, (s // k) % k, s // (k * k)])[:, None]
    delta = np.abs(co - sc)
    d = np.minimum(delta, k - delta).sum(axis=0)
    best = np.full(n, np.iinfo(np.int64).max)
    mult = np.array([1, k, k * k])
    for dim in range(3):
        for step in (1, k - 1):
            nco = co.copy()
            nco[dim] = (nco[dim] + step) % k
            u = (nco * mult[:, None]).sum(axis=0)
            ok = d[u] == d - 1
            best = np.where(ok, np.minimum(best, u), best)
    best[s] = s
    return d, best


@pytest.mark.parametrize("k", [3, 4, 5, 8, 16, 32])
def test_torus_closed_form(k):
    g = gg.torus3d(k)
    for s in gg.sources(g, 3, seed=3):
        d, p = oracle.bfs(g, int(s))
        ed, ep = torus_closed_form(k, int(s))
        assert np.array_equal(d, ed)
        assert np.array_equal(p, ep)


# ---------------------------------------------------------------------------
# Library routine, invariants, reductions
# ---------------------------------------------------------------------------

def _scipy_graph(g, weights):
    return sp.csr_matrix((weights.astype(np.float64), g.nbrs, g.offsets), shape=(g.n, g.n))


@pytest.mark.parametrize("scale", [8, 11])
def test_against_scipy_shortest_path(scale):
    g = gg.rmat(scale, seed=5)
    w = gg.weights(g, 24, seed=6)
    M = _scipy_graph(g, w)
    for s in gg.sources(g, 4, seed=7):
        s = int(s)
        d, p = oracle.bfs(g, s)
        ref = shortest_path(M, method="D", unweighted=True, indices=s)
        exp = np.where(np.isfinite(ref), ref, BFS_INF).astype(np.int64)
        assert np.array_equal(d, exp)
        d, p = oracle.wbfs(g, s, w)
        ref = shortest_path(M, method="D", indices=s)
        exp = np.where(np.isfinite(ref), ref, WBFS_INF).astype(np.int64)
        assert np.array_equal(d.astype(np.int64), exp)


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(14, seed=11),
    lambda: gg.erdos_renyi(1 << 13, 8, seed=12),
    lambda: gg.torus3d(20),
    lambda: gg.rmat(12, edge_factor=2, seed=13),  # many small components
])
def test_invariants_medium(make):
    g = make()
    g.weights = gg.weights(g, 24, seed=2)
    for s in gg.sources(g, 3, seed=3):
        s = int(s)
        d, p = oracle.bfs(g, s)
        check_bfs(g, s, d, p)
        d, p = oracle.wbfs(g, s)
        check_wbfs(g, s, d, p)


def test_unit_and_constant_weight_reductions():
    g = gg.rmat(12, seed=21)
    for s in gg.sources(g, 3, seed=3):
        s = int(s)
        db, pb = oracle.bfs(g, s)
        dw, pw = oracle.wbfs(g, s, np.ones(g.m, dtype=np.int32))
        reach = db != BFS_INF
        assert np.array_equal(dw[reach].astype(np.int64), db[reach])
        assert np.all(dw[~reach] == WBFS_INF)
        assert np.array_equal(pw, pb)
        dc, pc = oracle.wbfs(g, s, np.full(g.m, 7, dtype=np.int32))
        assert np.array_equal(dc[reach].astype(np.int64), 7 * db[reach].astype(np.int64))
        assert np.array_equal(pc, pb)


def test_checks_reject_plausible_mistakes():
    """Mutated oracle outputs (as a buggy implementation would produce) must
    fail the definition checks."""
    g = gg.rmat(11, seed=31)
    g.weights = gg.weights(g, 12, seed=32)
    s = int(gg.sources(g, 1, seed=3)[0])
    d, p = oracle.bfs(g, s)
    reach = np.nonzero((d != BFS_INF) & (np.arange(g.n) != s))[0]
    # 1. parent = max instead of min closer neighbour
    deg = g.degrees()
    for v in reach:
        nb = g.nbrs[g.offsets[v]:g.offsets[v + 1]]
        closer = nb[d[nb] == d[v] - 1]
        if len(closer) > 1:
            bad = p.copy()
            bad[v] = closer.max()
            with pytest.raises(AssertionError):
                check_bfs(g, s, d, bad)
            break
    # 2. off-by-one level on one vertex
    bad = d.copy()
    bad[reach[len(reach) // 2]] += 1
    with pytest.raises(AssertionError):
        check_bfs(g, s, bad, p)
    # 3. unreachable marked reachable
    unr = np.nonzero(d == BFS_INF)[0]
    if len(unr):
        bad = d.copy()
        bad[unr[0]] = 5
        with pytest.raises(AssertionError):
            check_bfs(g, s, bad, p)
    # 4. weighted: a distance one too large / parent ignoring the weight term
    dw, pw = oracle.wbfs(g, s)
    rw = np.nonzero((dw != WBFS_INF) & (np.arange(g.n) != s))[0]
    bad = dw.copy()
    bad[rw[3]] += 1
    with pytest.raises(AssertionError):
        check_wbfs(g, s, bad, pw)
    bad = dw.copy()
    bad[rw[5]] -= 1
    with pytest.raises(AssertionError):
        check_wbfs(g, s, bad, pw)
    # hop-count parent in place of weighted parent
    with pytest.raises(AssertionError):
        check_wbfs(g, s, dw, p)
    assert deg.sum() == g.m


def test_oracle_rejects_bad_arguments():
    g = gg.path(4)
    with pytest.raises(ValueError):
        oracle.bfs(g, 4)
    with pytest.raises(ValueError):
        oracle.bfs(g, -1)
    g.weights = np.array([1, 0, 0, 1, 1, 1], dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.wbfs(g, 0)
