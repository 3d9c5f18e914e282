"""GPU parity of general-weight SSSP (Bellman-Ford rounds) and widest path
against the oracle, element by element, through the C ABI."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

INF64 = int(oracle.SSSP_INF)
NEG64 = int(oracle.SSSP_NEG_INF)


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_05208_amd as m
    m.lib()
    return m


def _csr(n, und):
    edges = sorted([(u, v, w) for u, v, w in und] + [(v, u, w) for u, v, w in und])
    off = np.zeros(n + 1, dtype=np.int64)
    for u, _, _ in edges:
        off[u + 1] += 1
    g = gg.CSR(n=n, offsets=np.cumsum(off), nbrs=np.array([v for _, v, _ in edges], dtype=np.int32))
    g.weights = np.array([w for _, _, w in edges], dtype=np.int32)
    return g


def _first_bad(a, b):
    bad = np.nonzero(a != b)[0]
    return None if bad.size == 0 else (bad.size, int(bad[0]), a[bad[0]], b[bad[0]])


GRAPHS = {
    "rmat10": lambda: gg.rmat(10, seed=1),
    "rmat14": lambda: gg.rmat(14, seed=2),
    "rmat16": lambda: gg.rmat(16, seed=3),
    "rmat12_ef2": lambda: gg.rmat(12, edge_factor=2, seed=4),
    "er13": lambda: gg.erdos_renyi(1 << 13, 8, seed=5),
    "torus16": lambda: gg.torus3d(16),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("force", [0, 1, 2])
def test_parity_against_oracle(gb, name, force):
    g = GRAPHS[name]()
    w = gg.weights(g, 24, seed=7)
    G = gb.Graph(g.offsets, g.nbrs, w)
    opts = {"force_direction": force} if force else None
    for s in [int(x) for x in gg.sources(g, 3, seed=8)]:
        d = gb.bellman_ford(G, s, opts=opts).cpu().numpy()
        ref = oracle.bellman_ford(g, s, w)
        assert _first_bad(d, ref) is None, (name, force, s, _first_bad(d, ref))
        wd = gb.as_u32(gb.widest_path(G, s, opts=opts))
        wref = oracle.widest_path(g, s, w)
        assert _first_bad(wd, wref) is None, (name, force, s, _first_bad(wd, wref))
    G.free()


def test_stats_and_round_structure(gb):
    g = gg.rmat(14, seed=2)
    w = gg.weights(g, 24, seed=7)
    G = gb.Graph(g.offsets, g.nbrs, w)
    s = int(gg.sources(g, 1, seed=8)[0])
    d, st = gb.bellman_ford(G, s, stats=True)
    assert st["rounds"] >= 1 and st["launches"] >= st["rounds"]
    assert st["push_rounds"] + st["pull_rounds"] == st["rounds"]
    wd, st2 = gb.widest_path(G, s, stats=True)
    assert st2["rounds"] >= 1
    G.free()


def test_single_vertex_and_isolated_source(gb):
    g = gg.CSR(n=1, offsets=np.zeros(2, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    g.weights = np.zeros(0, dtype=np.int32)
    G = gb.Graph.from_csr(g)
    assert gb.bellman_ford(G, 0).cpu().tolist() == [0]
    assert gb.as_u32(gb.widest_path(G, 0)).tolist() == [0xFFFFFFFF]
    G.free()
    # an isolated source inside a larger graph
    und = [(1, 2, 3), (2, 3, 4)]
    g = _csr(5, und)
    G = gb.Graph.from_csr(g)
    assert gb.bellman_ford(G, 0).cpu().tolist() == [0] + [INF64] * 4
    assert gb.as_u32(gb.widest_path(G, 0)).tolist() == [0xFFFFFFFF, 0, 0, 0, 0]
    assert gb.as_u32(gb.widest_path(G, 1)).tolist() == [0, 0xFFFFFFFF, 3, 3, 0]
    G.free()


def test_unit_weights_give_bfs_distances(gb):
    g = gg.rmat(14, seed=9)
    ones = np.ones(g.m, dtype=np.int32)
    G = gb.Graph(g.offsets, g.nbrs, ones)
    for s in [int(x) for x in gg.sources(g, 2, seed=8)]:
        db, _ = gb.bfs(G, s)
        db = db.cpu().numpy().astype(np.int64)
        exp = np.where(db == 2**31 - 1, INF64, db)
        assert np.array_equal(gb.bellman_ford(G, s).cpu().numpy(), exp)
    G.free()


def test_zero_and_negative_weights(gb):
    # zero weights are fine for Bellman-Ford
    und = [(0, 1, 0), (1, 2, 0), (2, 3, 5), (0, 3, 7), (4, 5, 2)]
    g = _csr(6, und)
    G = gb.Graph.from_csr(g, signed_weights=True)
    assert gb.bellman_ford(G, 0).cpu().tolist() == list(oracle.bellman_ford(g, 0))
    G.free()
    # a negative edge in the source's component: the component is minus infinity
    und = [(0, 1, 4), (1, 2, -1), (2, 3, 2), (4, 5, 3), (5, 6, -2)]
    g = _csr(8, und)
    G = gb.Graph.from_csr(g, signed_weights=True)
    for s in range(8):
        assert gb.bellman_ford(G, s).cpu().tolist() == list(oracle.bellman_ford(g, s)), s
    G.free()
    # negative edges only outside the source's component: ordinary distances
    und = [(0, 1, 4), (1, 2, 1), (2, 3, 6), (4, 5, 3), (5, 6, -2)]
    g = _csr(8, und)
    G = gb.Graph.from_csr(g, signed_weights=True)
    d = gb.bellman_ford(G, 1).cpu().tolist()
    assert d == list(oracle.bellman_ford(g, 1)) == [4, 0, 1, 7] + [INF64] * 4
    # weights below 1 are refused by widest path and weighted BFS
    with pytest.raises(gb.GbgpuError):
        gb.widest_path(G, 0)
    with pytest.raises(gb.GbgpuError):
        gb.wbfs(G, 0)
    G.free()


def test_medium_graph_with_negative_weights(gb):
    """RMAT with a few negative edges planted symmetrically: the source's
    component is minus infinity when it holds one."""
    g = gg.rmat(12, edge_factor=2, seed=11)
    w = gg.weights(g, 16, seed=12).astype(np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    rng = np.random.default_rng(13)
    # plant negatives on a few undirected edges (both stored directions)
    und = np.nonzero(rows < g.nbrs)[0]
    pick = rng.choice(und, size=3, replace=False)
    for e in pick:
        u, v = rows[e], g.nbrs[e]
        back = g.offsets[v] + np.searchsorted(g.nbrs[g.offsets[v]:g.offsets[v + 1]], u)
        w[e] = w[back] = -5
    w = w.astype(np.int32)
    G = gb.Graph(g.offsets, g.nbrs, w, signed_weights=True)
    for s in [int(x) for x in gg.sources(g, 6, seed=14)]:
        d = gb.bellman_ford(G, s).cpu().numpy()
        ref = oracle.bellman_ford(g, s, w)
        assert _first_bad(d, ref) is None, (s, _first_bad(d, ref))
    G.free()


def test_weight_below_one_needs_the_signed_flag(gb):
    g = _csr(3, [(0, 1, 0), (1, 2, 2)])
    for validate in (True, False):
        with pytest.raises(gb.GbgpuError):
            gb.Graph.from_csr(g, validate=validate)
    G = gb.Graph.from_csr(g, signed_weights=True)
    assert gb.bellman_ford(G, 0).cpu().tolist() == [0, 0, 2]
    G.free()


def test_caller_stream_and_outputs(gb):
    g = gg.rmat(12, seed=15)
    w = gg.weights(g, 24, seed=7)
    G = gb.Graph(g.offsets, g.nbrs, w)
    s = int(gg.sources(g, 1, seed=8)[0])
    stream = torch.cuda.Stream()
    d = torch.full((g.n,), 7, dtype=torch.int64, device="cuda")
    wd = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(stream):
        gb.bellman_ford(G, s, dist=d, stream=stream)
        gb.widest_path(G, s, width=wd, stream=stream)
    stream.synchronize()
    assert np.array_equal(d.cpu().numpy(), oracle.bellman_ford(g, s, w))
    assert np.array_equal(gb.as_u32(wd), oracle.widest_path(g, s, w))
    G.free()
