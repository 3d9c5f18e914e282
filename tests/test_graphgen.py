"""Input generator checks (CPU): determinism, CSR well-formedness, weights,
sources.  The generator is shared by the oracle and the GPU path, so these
properties are what both sides rely on."""
import numpy as np
import pytest

import graphgen as gg


def assert_wellformed(g):
    off, nb = g.offsets, g.nbrs
    assert off.dtype == np.int64 and nb.dtype == np.int32
    assert off[0] == 0 and off[-1] == nb.size
    assert np.all(np.diff(off) >= 0)
    deg = np.diff(off)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    assert np.all(nb >= 0) and np.all(nb < g.n)
    assert not np.any(src == nb), "self loop"
    # strictly ascending within each list
    same = src[1:] == src[:-1]
    assert np.all(nb[1:][same] > nb[:-1][same]), "unsorted or duplicate"
    # symmetric: the multiset of (u, v) equals that of (v, u)
    a = np.sort(src * g.n + nb)
    b = np.sort(nb.astype(np.int64) * g.n + src)
    assert np.array_equal(a, b), "not symmetric"


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(10, seed=1),
    lambda: gg.rmat(13, edge_factor=4, seed=9),
    lambda: gg.erdos_renyi(3000, 10, seed=4),
    lambda: gg.torus3d(2),
    lambda: gg.torus3d(3),
    lambda: gg.torus3d(11),
    lambda: gg.grid2d(5, 7),
    lambda: gg.cycle(9),
])
def test_wellformed(make):
    assert_wellformed(make())


def test_rmat_deterministic_and_seeded():
    a = gg.rmat(12, seed=1)
    b = gg.rmat(12, seed=1)
    c = gg.rmat(12, seed=2)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.nbrs, b.nbrs)
    assert not (a.m == c.m and np.array_equal(a.nbrs, c.nbrs))


def test_rmat_thread_count_independent(monkeypatch):
    monkeypatch.setenv("GG_THREADS", "1")
    a = gg.rmat(12, seed=5)
    monkeypatch.setenv("GG_THREADS", "7")
    b = gg.rmat(12, seed=5)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.nbrs, b.nbrs)


def test_rmat_skew():
    g = gg.rmat(14, seed=1)
    deg = g.degrees()
    # RMAT (0.57, 0.19, 0.19, 0.05): heavy-tailed degrees, many isolated ids
    assert deg.max() > 50 * deg.mean()
    assert (deg == 0).sum() > g.n // 10


def test_torus_structure():
    k = 6
    g = gg.torus3d(k)
    assert g.n == k ** 3 and g.m == 6 * k ** 3
    v = 5 + k * 2 + k * k * 3
    nb = set(g.nbrs[g.offsets[v]:g.offsets[v + 1]].tolist())
    exp = {((v % k + dx) % k) + k * (((v // k) % k + dy) % k) + k * k * ((v // (k * k) + dz) % k)
           for dx, dy, dz in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]}
    assert nb == exp


def test_weights_symmetric_in_range():
    g = gg.rmat(11, seed=3)
    w = gg.weights(g, 24, seed=2)
    assert w.min() >= 1 and w.max() <= 23
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    key = src * g.n + g.nbrs
    rkey = g.nbrs.astype(np.int64) * g.n + src
    order = np.argsort(key)
    pos = np.searchsorted(key[order], rkey)
    assert np.array_equal(w, w[order][pos])
    # all values in [1, W) appear
    assert set(np.unique(w).tolist()) == set(range(1, 24))
    assert np.array_equal(w, gg.weights(g, 24, seed=2))


def test_sources_distinct_nonzero_degree():
    g = gg.rmat(12, seed=1)
    s = gg.sources(g, 64, seed=3)
    assert len(s) == 64 and len(set(s.tolist())) == 64
    assert np.all(g.degrees()[s] > 0)
    assert np.array_equal(s, gg.sources(g, 64, seed=3))
    assert np.array_equal(s[:16], gg.sources(g, 16, seed=3))


def test_relabel_preserves_structure():
    g = gg.rmat(9, seed=2)
    perm = np.random.default_rng(0).permutation(g.n)
    h = gg.relabel(g, perm)
    assert_wellformed(h)
    assert h.m == g.m
    assert np.array_equal(np.sort(h.degrees()), np.sort(g.degrees()))
