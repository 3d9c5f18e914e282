"""GPU parity of the low-diameter decomposition and of connectivity against
the oracle, through the C ABI.

Both are integer results: the clusters (centre ids) must equal the oracle's
bit for bit, since the shifts come from the same published generator and
ties go to the smallest claimer id on both sides; connectivity labels are the
smallest vertex id of each component on both sides.
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


GRAPHS = {
    "rmat10": lambda: gg.rmat(10, seed=1),
    "rmat14": lambda: gg.rmat(14, seed=2),
    "rmat16_ef4": lambda: gg.rmat(16, edge_factor=4, seed=3),
    "rmat13_ef2": lambda: gg.rmat(13, edge_factor=2, seed=4),
    "er14_d1": lambda: gg.erdos_renyi(1 << 14, 1, seed=5),
    "er13_d8": lambda: gg.erdos_renyi(1 << 13, 8, seed=6),
    "torus20": lambda: gg.torus3d(20),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_ldd_parity(gb, name):
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    for beta, seed in [(0.05, 1), (0.2, 7), (0.6, 2**63 + 5)]:
        cl, st = gb.ldd(G, beta, seed, stats=True)
        got = cl.cpu().numpy()
        exp = oracle.ldd(g, beta, seed)
        bad = np.nonzero(got != exp)[0]
        assert bad.size == 0, f"{name} beta={beta} seed={seed}: {bad.size} differ, first v={bad[0]} gpu={got[bad[0]]} oracle={exp[bad[0]]}"
        assert st["reached"] == int((exp == np.arange(g.n)).sum())
        gs = oracle.geo_shifts(g.n, beta, seed)
        assert st["rounds"] == int(gs.max()) + 1
    G.free()


@pytest.mark.parametrize("force", [1, 2])
@pytest.mark.parametrize("name", ["rmat14", "er13_d8", "torus20", "rmat13_ef2"])
def test_ldd_parity_each_direction(gb, name, force):
    """Every round sparse (push with atomic minimum) or every round dense
    (pull: first frontier neighbour in the sorted list): same clusters."""
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    for beta, seed in [(0.1, 5), (0.4, 6)]:
        got = gb.ldd(G, beta, seed, opts={"force_direction": force, "pull_light": 4}).cpu().numpy()
        assert np.array_equal(got, oracle.ldd(g, beta, seed)), f"{name} force={force} beta={beta}"
    assert np.array_equal(gb.connectivity(G, 0.3, 2, opts={"force_direction": force}).cpu().numpy(),
                          oracle.components(g))
    G.free()


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_connectivity_parity(gb, name):
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    exp = oracle.components(g)
    for beta, seed in [(0.2, 3), (0.5, 11)]:
        lab, st = gb.connectivity(G, beta, seed, stats=True)
        got = lab.cpu().numpy()
        bad = np.nonzero(got != exp)[0]
        assert bad.size == 0, f"{name} beta={beta}: {bad.size} differ, first v={bad[0]} gpu={got[bad[0]]} oracle={exp[bad[0]]}"
        assert st["reached"] == int(np.unique(exp).size)
        assert st["rounds"] >= 1
    G.free()


def test_edge_cases(gb):
    # a single vertex, no edges
    g = gg.CSR(n=1, offsets=np.zeros(2, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    G = gb.Graph.from_csr(g, with_weights=False)
    assert gb.ldd(G, 0.2, 1).cpu().tolist() == [0]
    lab, st = gb.connectivity(G, 0.2, 1, stats=True)
    assert lab.cpu().tolist() == [0] and st["reached"] == 1
    G.free()
    # no edges at all: every vertex is its own cluster and component
    n = 777
    g = gg.CSR(n=n, offsets=np.zeros(n + 1, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    G = gb.Graph.from_csr(g, with_weights=False)
    assert np.array_equal(gb.ldd(G, 0.3, 9).cpu().numpy(), np.arange(n))
    assert np.array_equal(gb.connectivity(G, 0.3, 9).cpu().numpy(), np.arange(n))
    G.free()
    # a long path (many LDD rounds and levels), a ring, cliques side by side
    n = 3000
    for und in ([(i, i + 1) for i in range(n - 1)],
                [(i, (i + 1) % n) for i in range(n)],
                [(b + u, b + v) for b in range(0, 60, 6) for u in range(6) for v in range(u + 1, 6)]):
        g = _csr_und(n, und)
        G = gb.Graph.from_csr(g)
        for beta, seed in [(0.1, 4), (0.9, 5)]:
            assert np.array_equal(gb.ldd(G, beta, seed).cpu().numpy(), oracle.ldd(g, beta, seed))
            assert np.array_equal(gb.connectivity(G, beta, seed).cpu().numpy(), oracle.components(g))
        G.free()


def test_independent_of_beta_and_seed_and_repeatable(gb):
    g = gg.rmat(15, edge_factor=2, seed=8)
    G = gb.Graph.from_csr(g)
    exp = oracle.components(g)
    for beta, seed in [(0.01, 0), (0.3, 1), (0.99, 2**64 - 1), (0.3, 1)]:
        assert np.array_equal(gb.connectivity(G, beta, seed).cpu().numpy(), exp)
    a = gb.ldd(G, 0.25, 42).cpu().numpy()
    b = gb.ldd(G, 0.25, 42).cpu().numpy()
    assert np.array_equal(a, b)
    G.free()


def test_many_distinct_cross_edges(gb):
    """Small clusters on a 128^3 torus (beta 0.95): 1.3 million distinct
    inter-cluster edges, more than the first key buffer holds (the cross
    pass runs again with room for all of them)."""
    g = gg.torus3d(128)
    G = gb.Graph.from_csr(g, validate=False, with_weights=False)
    exp = oracle.components(g)
    for beta in (0.95, 0.5):
        assert np.array_equal(gb.ldd(G, beta, 17).cpu().numpy(), oracle.ldd(g, beta, 17))
        lab, st = gb.connectivity(G, beta, 17, stats=True)
        assert np.array_equal(lab.cpu().numpy(), exp), f"beta={beta}"
        assert st["reached"] == int(np.unique(exp).size)
    G.free()


def test_bad_beta(gb):
    g = gg.rmat(8, seed=1)
    G = gb.Graph.from_csr(g)
    for beta in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(gb.GbgpuError):
            gb.ldd(G, beta, 1)
        with pytest.raises(gb.GbgpuError):
            gb.connectivity(G, beta, 1)
    G.free()
