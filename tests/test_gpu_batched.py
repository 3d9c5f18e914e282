"""GPU parity for batched traversal: multi-source BFS (bit-packed frontiers)
and the uneven multi-graph batch must equal the oracle row by row, and the
single-source GPU path."""
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


def check_rows(g, srcs, D, P, tag=""):
    D = D.cpu().numpy()
    P = P.cpu().numpy()
    for i, s in enumerate(srcs):
        od, op = oracle.bfs(g, int(s))
        bad = np.nonzero((D[i] != od) | (P[i] != op))[0]
        assert bad.size == 0, (f"{tag} row {i} src {s}: {bad.size} mismatches, v={bad[0]} "
                               f"gpu ({D[i][bad[0]]},{P[i][bad[0]]}) oracle ({od[bad[0]]},{op[bad[0]]})")


@pytest.fixture(scope="module")
def rmat14(gb):
    g = gg.rmat(14, seed=21)
    return g, gb.Graph.from_csr(g)


@pytest.mark.parametrize("k", [1, 7, 64, 65, 130])
def test_multi_source_matches_oracle(gb, rmat14, k):
    g, G = rmat14
    srcs = gg.sources(g, k, seed=3)
    D, P = gb.bfs_multi(G, srcs)
    check_rows(g, srcs, D, P, tag=f"k={k}")


def test_multi_source_repeats_and_isolated(gb, rmat14):
    g, G = rmat14
    s = gg.sources(g, 5, seed=4)
    iso = int(np.nonzero(g.degrees() == 0)[0][0])
    srcs = np.array([s[0], s[1], s[0], iso, s[2], s[2], s[3]], dtype=np.int32)
    D, P = gb.bfs_multi(G, srcs)
    check_rows(g, srcs, D, P, tag="repeats")


@pytest.mark.parametrize("force", [1, 2])
def test_multi_source_forced_directions(gb, rmat14, force):
    g, G = rmat14
    srcs = gg.sources(g, 40, seed=5)
    D, P = gb.bfs_multi(G, srcs, opts={"force_direction": force})
    check_rows(g, srcs, D, P, tag=f"force{force}")


def test_multi_source_equals_single_source_path(gb):
    g = gg.rmat(16, seed=1)
    G = gb.Graph.from_csr(g)
    srcs = gg.sources(g, 64, seed=3)
    D, P = gb.bfs_multi(G, srcs)
    for i in (0, 17, 63):
        d, p = gb.bfs(G, int(srcs[i]))
        assert torch.equal(d, D[i]) and torch.equal(p, P[i])
    check_rows(g, srcs[:8], D[:8], P[:8], tag="rmat16")


def test_multi_source_torus_and_small(gb):
    for g in (gg.torus3d(10), gg.cycle(12), gg.path(3), gg.star(5)):
        G = gb.Graph.from_csr(g)
        srcs = np.arange(min(g.n, 70), dtype=np.int32) % g.n
        D, P = gb.bfs_multi(G, srcs)
        check_rows(g, srcs, D, P, tag=g.name)


def test_uneven_multi_graph_batch(gb):
    scales = [8, 9, 10, 11, 12, 13, 14, 10]
    graphs = [gg.rmat(s, seed=30 + i) for i, s in enumerate(scales)]
    Gs = [gb.Graph.from_csr(g) for g in graphs]
    qg, qs = [], []
    for i, g in enumerate(graphs):
        for s in gg.sources(g, 32 if i != 3 else 70, seed=40 + i):
            qg.append(i)
            qs.append(int(s))
    rng = np.random.default_rng(0)
    order = rng.permutation(len(qg))
    qg = [qg[i] for i in order]
    qs = [qs[i] for i in order]
    dists, parents = gb.bfs_batch([Gs[i] for i in qg], qs)
    for q in range(len(qg)):
        od, op = oracle.bfs(graphs[qg[q]], qs[q])
        assert np.array_equal(dists[q].cpu().numpy(), od), q
        assert np.array_equal(parents[q].cpu().numpy(), op), q


def test_batch_argument_errors(gb, rmat14):
    g, G = rmat14
    with pytest.raises(gb.GbgpuError):
        gb.bfs_multi(G, [g.n])
    with pytest.raises(gb.GbgpuError):
        gb.bfs_multi(G, [])


def test_deep_graphs_batched(gb):
    """Graphs a single-source BFS has shown to be deep are batched like any
    other: the 300-cycle (151 levels) with 4-byte pair entries, the
    600-cycle (301 levels, more than the 8-bit round field holds) with
    8-byte entries from the start; mixed with a shallow graph in one batch.
    Results equal the oracle."""
    deep, shallow = gg.cycle(300), gg.rmat(10, seed=5)
    Gd, Gs = gb.Graph.from_csr(deep), gb.Graph.from_csr(shallow)
    d0, p0, st = gb.bfs(Gd, 0, stats=True)
    assert st["rounds"] == 151
    srcs = [0, 17, 150, 299]
    D, P = gb.bfs_multi(Gd, srcs)
    check_rows(deep, srcs, D, P, tag="deep multi")
    deeper = gg.cycle(600)
    Gdd = gb.Graph.from_csr(deeper)
    _, _, st = gb.bfs(Gdd, 0, stats=True)
    assert st["rounds"] == 301
    srcs = [0, 1, 300, 599, 0]
    D, P = gb.bfs_multi(Gdd, srcs)
    check_rows(deeper, srcs, D, P, tag="deeper multi")
    Gdd.free()
    ss = [int(x) for x in gg.sources(shallow, 3, seed=2)]
    graphs = [deep, shallow, deep, shallow, shallow]
    qg = [Gd, Gs, Gd, Gs, Gs]
    qs = [3, ss[0], 200, ss[1], ss[2]]
    dists, parents = gb.bfs_batch(qg, qs)
    for q, (h, s) in enumerate(zip(graphs, qs)):
        od, op = oracle.bfs(h, s)
        assert np.array_equal(dists[q].cpu().numpy(), od), q
        assert np.array_equal(parents[q].cpu().numpy(), op), q


@pytest.mark.parametrize("persistent", [0, 1])
def test_batched_rounds_past_the_narrow_round_field(gb, persistent):
    """A group on a graph of at most 2^24 vertices keeps each (vertex,
    source) pair in 4 bytes with an 8-bit round of arrival.  Fresh handles
    (depth unknown, so the sources are batched): a 255-vertex path from one
    end reaches distance 254 within the field; a 256-vertex path and a
    1200-cycle run past round 254, stop, and the call runs again with 8-byte
    entries, also for the shallow graph batched beside them.  Every row
    equals the oracle."""
    opts = {"persistent": persistent}
    for n in (255, 256):
        h = gg.path(n)
        G = gb.Graph.from_csr(h)
        srcs = [0, n - 1, n // 2, 0]
        D, P = gb.bfs_multi(G, srcs, opts=opts)
        check_rows(h, srcs, D, P, tag=f"path{n}")
        assert int(D[0].max()) == n - 1
        G.free()
    deep, shallow = gg.cycle(1200), gg.rmat(10, seed=5)
    Gd, Gs = gb.Graph.from_csr(deep), gb.Graph.from_csr(shallow)
    ss = [int(x) for x in gg.sources(shallow, 3, seed=2)]
    graphs = [deep, shallow, deep, shallow, shallow]
    qg = [Gd, Gs, Gd, Gs, Gs]
    qs = [3, ss[0], 700, ss[1], ss[2]]
    dists, parents = gb.bfs_batch(qg, qs, opts=opts)
    for q, (h, s) in enumerate(zip(graphs, qs)):
        od, op = oracle.bfs(h, s)
        assert np.array_equal(dists[q].cpu().numpy(), od), q
        assert np.array_equal(parents[q].cpu().numpy(), op), q
    Gd.free()
    Gs.free()


def sparse_csr(n, edges, name):
    """Symmetric CSR of a few undirected edges over n vertices (numpy only,
    for n in the millions)."""
    e = np.asarray(edges, dtype=np.int64)
    us = np.concatenate([e[:, 0], e[:, 1]])
    vs = np.concatenate([e[:, 1], e[:, 0]])
    order = np.lexsort((vs, us))
    us, vs = us[order], vs[order]
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offsets, us + 1, 1)
    return gg.CSR(n=n, offsets=np.cumsum(offsets), nbrs=vs.astype(np.int32), name=name)


@pytest.mark.parametrize("n", [1 << 24, (1 << 24) + 1])
def test_batched_parents_at_the_24_bit_limit(gb, n):
    """4-byte pair entries keep a 24-bit parent: with n = 2^24 (the largest
    graph that uses them) vertex 2^24 - 1 is a hub and a parent; with
    n = 2^24 + 1 the entries are 8 bytes and vertex 2^24 is a parent.  A few
    edges among low and high ids; every row equals the oracle."""
    top = n - 1
    edges = [(0, 1), (1, 2), (2, 3), (top, 0), (top, top - 1), (top, 7), (top - 1, 5), (5, 6),
             (3, 4), (top - 2, top - 1)]
    h = sparse_csr(n, edges, f"sparse{n}")
    G = gb.Graph.from_csr(h, with_weights=False)
    srcs = [top, 3, top - 1, 6, 0]
    D, P = gb.bfs_multi(G, srcs)
    check_rows(h, srcs, D, P, tag=f"n={n}")
    assert int(P[1][top]) == 0 and int(P[3][7]) == top
    del D, P
    G.free()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("join_round", [0, 5, 9, 40])
def test_sources_joining_a_running_group(gb, rmat14, join_round):
    """Round-boundary admission: srcs[:5] start a packed group, the rest join
    it at a later round (before the group has finished, or after it ran out
    of work: join_round 40), with a repeated source among the joiners and a
    joiner equal to a starting source.  Every row equals the oracle."""
    g, G = rmat14
    srcs = [int(x) for x in gg.sources(g, 12, seed=7)]
    srcs = srcs[:5] + srcs[5:11] + [srcs[6], srcs[0]]
    D, P = gb.bfs_join(G, srcs, 5, join_round)
    check_rows(g, srcs, D, P, tag=f"join at {join_round}")


def test_joining_on_deep_and_small_graphs(gb):
    for g, k0, jr in ((gg.cycle(100), 2, 20), (gg.torus3d(8), 30, 4), (gg.path(7), 1, 0)):
        G = gb.Graph.from_csr(g, with_weights=False)
        srcs = (np.arange(min(g.n, 64), dtype=np.int32) * 7 + 3) % g.n
        D, P = gb.bfs_join(G, srcs, k0, jr)
        check_rows(g, srcs, D, P, tag=f"{g.name} join at {jr}")
        G.free()


@pytest.mark.parametrize("k", [1, 7, 64, 130])
def test_single_launch_batches_match_oracle(gb, rmat14, k):
    """Every round of every group in one cooperative launch (grid barriers
    between rounds, groups dropping out as their frontiers empty): the same
    rows as the oracle, in one launch."""
    g, G = rmat14
    srcs = gg.sources(g, k, seed=3)
    D, P, st = gb.bfs_multi(G, srcs, opts={"persistent": 1}, stats=True)
    check_rows(g, srcs, D, P, tag=f"single launch k={k}")
    assert st["launches"] == 1, st


@pytest.mark.parametrize("force", [1, 2])
def test_single_launch_batches_forced_directions(gb, rmat14, force):
    g, G = rmat14
    srcs = gg.sources(g, 40, seed=5)
    D, P = gb.bfs_multi(G, srcs, opts={"persistent": 1, "force_direction": force, "grid": 37})
    check_rows(g, srcs, D, P, tag=f"single launch force{force}")


def test_single_launch_uneven_batch_and_small_graphs(gb):
    """The uneven multi-graph batch in one launch (groups of different
    graphs finishing at different rounds), and small graphs whose grid is a
    single workgroup."""
    scales = [8, 9, 10, 11, 12, 13, 14, 10]
    graphs = [gg.rmat(s, seed=30 + i) for i, s in enumerate(scales)]
    Gs = [gb.Graph.from_csr(g) for g in graphs]
    qg, qs = [], []
    for i, g in enumerate(graphs):
        for s in gg.sources(g, 32 if i != 3 else 70, seed=40 + i):
            qg.append(i)
            qs.append(int(s))
    dists, parents, st = gb.bfs_batch([Gs[i] for i in qg], qs, opts={"persistent": 1},
                                      stats=True)
    for q in range(len(qg)):
        od, op = oracle.bfs(graphs[qg[q]], qs[q])
        assert np.array_equal(dists[q].cpu().numpy(), od), q
        assert np.array_equal(parents[q].cpu().numpy(), op), q
    assert st["launches"] >= 1
    for g in (gg.torus3d(10), gg.cycle(12), gg.path(3), gg.star(5)):
        G = gb.Graph.from_csr(g)
        srcs = np.arange(min(g.n, 70), dtype=np.int32) % g.n
        D, P = gb.bfs_multi(G, srcs, opts={"persistent": 1})
        check_rows(g, srcs, D, P, tag=f"single launch {g.name}")


def test_single_launch_batches_many_workgroups(gb):
    g = gg.rmat(16, seed=2)
    G = gb.Graph.from_csr(g, with_weights=False)
    srcs = gg.sources(g, 100, seed=6)
    D, P, st = gb.bfs_multi(G, srcs, opts={"persistent": 1, "grid": 512}, stats=True)
    check_rows(g, srcs[::9], D[::9], P[::9], tag="single launch grid 512")
    D2, P2 = gb.bfs_multi(G, srcs)
    assert torch.equal(D, D2) and torch.equal(P, P2)
    assert st["launches"] == 1
    G.free()
