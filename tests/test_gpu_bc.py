"""GPU parity of single-source betweenness against the oracle, through the
C ABI.

Tolerance: path counts and dependencies are sums of positive fp64 terms.  A
level's sums add at most (max degree) * 2^-53 relative error to what they
add up, the dependencies carry the counts' error plus their own, so either
side is within 2 * levels * max_degree * 2^-53 of the exact value and the
two within twice that; the tests allow twice that again.  Zeros (the
source, vertices without children, unreachable vertices) are exact on both
sides.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_05208_amd as m
    m.lib()
    return m


def _csr_und(n, und):
    edges = sorted(set([(u, v) for u, v in und] + [(v, u) for u, v in und]))
    off = np.zeros(n + 1, dtype=np.int64)
    for u, _ in edges:
        off[u + 1] += 1
    return gg.CSR(n=n, offsets=np.cumsum(off), nbrs=np.array([v for _, v in edges], dtype=np.int32))


def rtol_for(g, levels):
    maxdeg = int(np.diff(g.offsets).max()) if g.m else 1
    return 8.0 * max(levels, 1) * max(maxdeg, 1) * 2.0 ** -53


def oracle_levels(g, src):
    """Number of BFS levels from src, from the oracle's distances (the
    tolerance never takes a figure the device reported)."""
    d, _ = oracle.bfs(g, src)
    return int(d[d != oracle.BFS_INF].max()) + 1


def assert_close(got, exp, rtol, tag):
    assert np.array_equal(got == 0, exp == 0), f"{tag}: zero pattern differs"
    rel = np.abs(got - exp) / np.maximum(np.abs(exp), 1e-300)
    worst = int(np.argmax(rel))
    assert rel[worst] <= rtol, f"{tag}: v={worst} gpu={got[worst]!r} oracle={exp[worst]!r} rel={rel[worst]:.3g} > {rtol:.3g}"


GRAPHS = {
    "rmat10": lambda: gg.rmat(10, seed=1),
    "rmat14": lambda: gg.rmat(14, seed=2),
    "rmat16": lambda: gg.rmat(16, seed=3),
    "rmat12_ef2": lambda: gg.rmat(12, edge_factor=2, seed=4),
    "er13": lambda: gg.erdos_renyi(1 << 13, 8, seed=5),
    "torus16": lambda: gg.torus3d(16),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_parity_against_oracle(gb, name):
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    for s in [int(x) for x in gg.sources(g, 3, seed=8)]:
        dep, st = gb.betweenness(G, s, stats=True)
        exp = oracle.betweenness(g, s)
        levels = oracle_levels(g, s)
        assert_close(dep.cpu().numpy(), exp, rtol_for(g, levels), f"{name} src={s}")
        d, _ = oracle.bfs(g, s)
        reach = d != oracle.BFS_INF
        assert st["reached"] == int(reach.sum())
        assert st["rounds"] == levels
    G.free()


def test_closed_forms(gb):
    n = 9
    path = _csr_und(n, [(i, i + 1) for i in range(n - 1)])
    G = gb.Graph.from_csr(path)
    assert gb.betweenness(G, 0).cpu().tolist() == [0.0] + [float(n - 1 - v) for v in range(1, n)]
    G.free()
    c8 = _csr_und(8, [(i, (i + 1) % 8) for i in range(8)])
    G = gb.Graph.from_csr(c8)
    assert gb.betweenness(G, 0).cpu().tolist() == [0, 2.5, 1.5, 0.5, 0, 0.5, 1.5, 2.5]
    G.free()
    star = _csr_und(7, [(0, k) for k in range(1, 7)])
    G = gb.Graph.from_csr(star)
    assert gb.betweenness(G, 0).cpu().tolist() == [0.0] * 7
    assert gb.betweenness(G, 3).cpu().tolist() == [5.0] + [0.0] * 6
    G.free()


def test_single_vertex_and_isolated_source(gb):
    g = gg.CSR(n=1, offsets=np.zeros(2, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    G = gb.Graph.from_csr(g, with_weights=False)
    dep, st = gb.betweenness(G, 0, stats=True)
    assert dep.cpu().tolist() == [0.0] and st["rounds"] == 1 and st["reached"] == 1
    G.free()
    g = _csr_und(6, [(1, 2), (2, 3), (3, 4)])
    G = gb.Graph.from_csr(g)
    assert gb.betweenness(G, 0).cpu().tolist() == [0.0] * 6
    assert gb.betweenness(G, 1).cpu().tolist() == [0.0, 0.0, 2.0, 1.0, 0.0, 0.0]
    G.free()


def test_sum_identity_and_repeat(gb):
    """sum_v S[v] = sum over reachable t != src of (d(src, t) - 1); a second
    call on the same graph (workspace reuse) gives the same sums."""
    g = gg.rmat(15, seed=21)
    G = gb.Graph.from_csr(g)
    for s in [int(x) for x in gg.sources(g, 2, seed=3)]:
        d, _ = gb.bfs(G, s)
        d = d.cpu().numpy().astype(np.int64)
        reach = (d != 2**31 - 1) & (np.arange(g.n) != s)
        want = float((d[reach] - 1).sum())
        a = gb.betweenness(G, s).cpu().numpy()
        b = gb.betweenness(G, s).cpu().numpy()
        assert np.isclose(a.sum(), want, rtol=1e-9) and np.isclose(b.sum(), want, rtol=1e-9)
    G.free()
