"""Compressed adjacency on the GPU, through the C ABI: the compressed copy
decodes back to the graph's own neighbour array (bit-exact), and the BFS
that reads only the compressed lists, as well as the same rounds over the
plain lists, return the oracle's distances and min-ID parents exactly, in
every direction mode.
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
    "rmat16": lambda: gg.rmat(16, seed=3),
    "rmat13_ef2": lambda: gg.rmat(13, edge_factor=2, seed=4),
    "er13_d8": lambda: gg.erdos_renyi(1 << 13, 8, seed=5),
    "torus16": lambda: gg.torus3d(16),
    # a hub of degree 6000: a block table of 94 entries (more than one
    # wavefront's worth of blocks)
    "star6000": lambda: _csr_und(6001, [(0, k) for k in range(1, 6001)] + [(k, k + 1) for k in range(1, 6000, 7)]),
}


def _words_bytes(g):
    deg = np.diff(g.offsets)
    words = 0
    for v in range(g.n):
        d = int(deg[v])
        nb = (d + 63) // 64
        words += nb if nb > 1 else 0
        for k in range(nb):
            s = int(g.offsets[v]) + 64 * k
            ln = min(64, d - 64 * k)
            w = int(int(g.nbrs[s + ln - 1]) - int(g.nbrs[s])).bit_length()
            words += 2 + (ln * w + 31) // 32
    return 4 * words + 8 * (g.n + 1)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_round_trip_and_size(gb, name):
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    nbytes = gb.compress(G)
    assert nbytes == _words_bytes(g)
    got = gb.decompress(G).cpu().numpy()
    assert np.array_equal(got, g.nbrs)
    G.free()


@pytest.mark.parametrize("force", [0, 1, 2])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_bfs_parity(gb, name, force):
    g = GRAPHS[name]()
    G = gb.Graph.from_csr(g)
    gb.compress(G)
    opts = {"force_direction": force, "pull_light": 8} if force else None
    for s in [int(x) for x in gg.sources(g, 3, seed=9)]:
        ed, ep = oracle.bfs(g, s)
        reach = ed != oracle.BFS_INF
        for fn in (gb.bfs_compressed, gb.bfs_simple):
            d, p, st = fn(G, s, opts=opts, stats=True)
            d = d.cpu().numpy()
            p = p.cpu().numpy()
            bad = np.nonzero((d != ed) | (p != ep))[0]
            assert bad.size == 0, (f"{name} {fn.__name__} force={force} src={s}: {bad.size} differ, "
                                   f"first v={bad[0]} gpu=({d[bad[0]]},{p[bad[0]]}) "
                                   f"oracle=({ed[bad[0]]},{ep[bad[0]]})")
            assert st["reached"] == int(reach.sum())
            assert st["rounds"] == int(ed[reach].max()) + 1
    G.free()


def test_edge_cases(gb):
    # one vertex, no edges
    g = gg.CSR(n=1, offsets=np.zeros(2, dtype=np.int64), nbrs=np.zeros(0, dtype=np.int32))
    G = gb.Graph.from_csr(g, with_weights=False)
    assert gb.compress(G) == 16
    d, p = gb.bfs_compressed(G, 0)
    assert d.cpu().tolist() == [0] and p.cpu().tolist() == [0]
    G.free()
    # isolated source on a graph with edges; a path (one vertex per round)
    g = _csr_und(500, [(i, i + 1) for i in range(1, 499)])
    G = gb.Graph.from_csr(g)
    gb.compress(G)
    for s in (0, 1, 250):
        ed, ep = oracle.bfs(g, s)
        d, p = gb.bfs_compressed(G, s)
        assert np.array_equal(d.cpu().numpy(), ed) and np.array_equal(p.cpu().numpy(), ep)
    G.free()


def test_needs_a_compressed_copy(gb):
    g = gg.rmat(8, seed=1)
    G = gb.Graph.from_csr(g)
    with pytest.raises(gb.GbgpuError):
        gb.bfs_compressed(G, 0)
    with pytest.raises(gb.GbgpuError):
        gb.decompress(G)
    d, p = gb.bfs_simple(G, int(gg.sources(g, 1, seed=1)[0]))   # no copy needed
    with pytest.raises(gb.GbgpuError):
        gb.bfs_compressed(G, g.n)                                  # bad source checked first
    gb.compress(G)
    gb.compress(G)                                                 # rebuilding is allowed
    assert np.array_equal(gb.decompress(G).cpu().numpy(), g.nbrs)
    G.free()
