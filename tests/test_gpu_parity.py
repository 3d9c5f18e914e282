"""GPU parity: libgbgpu BFS / weighted BFS against the oracle, element by
element (integer outputs: bit-exact distances and min-ID parents)."""
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


def run_bfs(gb, G, src, opts=None):
    d, p = gb.bfs(G, src, opts=opts)
    return d.cpu().numpy(), p.cpu().numpy()


def run_wbfs(gb, G, src, opts=None):
    d, p = gb.wbfs(G, src, opts=opts)
    return gb.as_u32(d), p.cpu().numpy()


def assert_bfs(gb, g, G, src, opts=None, tag=""):
    d, p = run_bfs(gb, G, src, opts)
    od, op = oracle.bfs(g, src)
    bad = np.nonzero((d != od) | (p != op))[0]
    assert bad.size == 0, (f"{tag} src={src}: {bad.size} mismatches, first v={bad[0]}: "
                           f"gpu ({d[bad[0]]},{p[bad[0]]}) oracle ({od[bad[0]]},{op[bad[0]]})")


def assert_wbfs(gb, g, G, src, opts=None, tag=""):
    d, p = run_wbfs(gb, G, src, opts)
    od, op = oracle.wbfs(g, src)
    bad = np.nonzero((d != od) | (p != op))[0]
    assert bad.size == 0, (f"{tag} src={src}: {bad.size} mismatches, first v={bad[0]}: "
                           f"gpu ({d[bad[0]]},{p[bad[0]]}) oracle ({od[bad[0]]},{op[bad[0]]})")


def small_graphs():
    out = [gg.path(1), gg.path(2), gg.path(17), gg.cycle(10), gg.cycle(11), gg.star(70),
           gg.complete(9), gg.grid2d(13, 7), gg.torus3d(3), gg.torus3d(6)]
    rng = np.random.default_rng(5)
    for _ in range(12):
        n = int(rng.integers(2, 40))
        A = np.triu(rng.random((n, n)) < rng.uniform(0.05, 0.5), 1)
        u, v = np.nonzero(A)
        out.append(gg.from_edges(n, list(zip(u, v))))
    return out


def test_small_graphs_all_sources(gb):
    rng = np.random.default_rng(9)
    for g in small_graphs():
        g.weights = gg.weights(g, 6, seed=4) if g.m else np.zeros(0, np.int32)
        G = gb.Graph.from_csr(g)
        for s in range(g.n):
            assert_bfs(gb, g, G, s, tag=g.name)
            if g.m:
                assert_wbfs(gb, g, G, s, tag=g.name)
                for force in (2, 3):
                    assert_wbfs(gb, g, G, s, opts={"force_direction": force},
                                tag=f"{g.name} wforce{force}")
        G.free()


def test_golden_fixtures(gb):
    import os
    from test_oracle import _parse_golden, _vals
    for name in ("small_unweighted.txt", "small_weighted.txt"):
        g, src, rows = _parse_golden(name)
        G = gb.Graph.from_csr(g)
        d, p = run_bfs(gb, G, src)
        assert np.array_equal(d.astype(np.int64), _vals(rows["bfs_dist"], 2**31 - 1))
        assert np.array_equal(p.astype(np.int64), _vals(rows["bfs_parent"], -1))
        if "wbfs_dist" in rows:
            d, p = run_wbfs(gb, G, src)
            assert np.array_equal(d.astype(np.int64), _vals(rows["wbfs_dist"], 0xFFFFFFFF))
            assert np.array_equal(p.astype(np.int64), _vals(rows["wbfs_parent"], -1))


@pytest.fixture(scope="module")
def rmat16(gb):
    g = gg.rmat(16, seed=1).with_weights(24, seed=2)
    return g, gb.Graph.from_csr(g)


def test_rmat16_bfs_sources(gb, rmat16):
    g, G = rmat16
    for s in gg.sources(g, 16, seed=3):
        assert_bfs(gb, g, G, int(s), tag="rmat16")


def test_rmat16_wbfs_sources(gb, rmat16):
    g, G = rmat16
    for s in gg.sources(g, 8, seed=3):
        assert_wbfs(gb, g, G, int(s), tag="rmat16")


@pytest.mark.parametrize("force", [1, 2, 3])
def test_forced_directions_identical(gb, rmat16, force):
    g, G = rmat16
    for s in gg.sources(g, 4, seed=3):
        assert_bfs(gb, g, G, int(s), opts={"force_direction": force}, tag=f"force{force}")


@pytest.mark.parametrize("force", [1, 2, 3])
def test_wbfs_forced_directions_identical(gb, rmat16, force):
    g, G = rmat16
    for s in gg.sources(g, 4, seed=3):
        assert_wbfs(gb, g, G, int(s), opts={"force_direction": force}, tag=f"wforce{force}")


def test_wbfs_bucket_peak(gb, rmat16):
    """bucket_peak is the largest entry count of the buckets the search
    processed (their fill, what the capacity must hold): the largest count
    in the step log, and never above the capacity of a run that did not
    have to grow it."""
    g, G = rmat16
    for s in (int(x) for x in gg.sources(g, 3, seed=5)):
        for opts in (None, {"bucket_capacity": 64}):
            _, _, st = gb.wbfs(G, s, opts=opts, stats=True)
            lg = G.wbfs_log()
            assert st["bucket_peak"] == int(lg[lg[:, 3] != 2, 1].max()) > 0
            if opts:
                assert st["bucket_peak"] <= min(g.n, 64 * 2 ** st["retries"]), st


def test_wbfs_dense_steps_in_auto_mode(gb, rmat16):
    """The default threshold sends the heavy buckets of an RMAT graph dense;
    every dense bucket takes a marking launch followed by a pull launch of
    the same bucket, and buckets come out in increasing order."""
    g, G = rmat16
    s = int(gg.sources(g, 1, seed=3)[0])
    d, p, st = gb.wbfs(G, s, stats=True)
    assert st["pull_rounds"] > 0 and st["push_rounds"] > 0
    lg = G.wbfs_log()
    kinds = lg[:, 3]
    assert set(np.unique(kinds)) <= {0, 1, 2}
    for i in np.nonzero(kinds == 1)[0]:
        assert kinds[i + 1] == 2 and lg[i + 1, 0] == lg[i, 0]
    buckets = lg[kinds != 2, 0]
    assert np.all(np.diff(buckets.astype(np.int64)) > 0)
    assert st["rounds"] == len(buckets) and st["pull_rounds"] == int((kinds == 2).sum())
    od, op = oracle.wbfs(g, s)
    assert np.array_equal(gb.as_u32(d), od) and np.array_equal(p.cpu().numpy(), op)


@pytest.mark.parametrize("opts", [
    {"wave_chunk": 64}, {"wave_chunk": 256, "grid": 7}, {"grid": 1}, {"grid": 3, "pull_light": 1},
    {"pull_light": 4, "tau": 2}, {"tau": 1000}, {"rounds_per_sync": 1},
    {"beta": -1}, {"beta": 2, "tau": 4}, {"beta": 100000},
])
def test_tuning_knobs_identical(gb, rmat16, opts):
    g, G = rmat16
    for s in gg.sources(g, 3, seed=3):
        assert_bfs(gb, g, G, int(s), opts=opts, tag=str(opts))
        assert_wbfs(gb, g, G, int(s), opts=opts, tag=str(opts))


@pytest.mark.parametrize("opts", [{"bucket_capacity": 64}, {"bucket_window": 256},
                                  {"bucket_capacity": 1000, "grid": 5}])
def test_bucket_knobs_identical(gb, rmat16, opts):
    g, G = rmat16
    for s in gg.sources(g, 2, seed=3):
        assert_wbfs(gb, g, G, int(s), opts=opts, tag=str(opts))


def test_repeat_runs_identical(gb, rmat16):
    g, G = rmat16
    s = int(gg.sources(g, 1, seed=3)[0])
    d0, p0 = run_bfs(gb, G, s)
    w0, q0 = run_wbfs(gb, G, s)
    for _ in range(5):
        d, p = run_bfs(gb, G, s)
        assert np.array_equal(d, d0) and np.array_equal(p, p0)
        w, q = run_wbfs(gb, G, s)
        assert np.array_equal(w, w0) and np.array_equal(q, q0)


@pytest.mark.parametrize("ahead", [1, 3, 8])
def test_round_log_and_stats(gb, rmat16, ahead):
    """The round log holds one entry per non-empty frontier of this call over
    the vertices of degree >= 2 (a run with fewer rounds after a longer one
    must not show stale entries), whatever the launch look-ahead; degree-1
    vertices are attached after the last round and counted in the stats."""
    g, G = rmat16
    INF = 2**31 - 1
    cyc = gg.cycle(40).with_weights(6, seed=4)
    C = gb.Graph.from_csr(cyc)
    for GG, gg_, s in ((G, g, int(gg.sources(g, 1, seed=3)[0])), (C, cyc, 0),
                       (G, g, int(gg.sources(g, 2, seed=5)[1]))):
        d, p, st = gb.bfs(GG, s, opts={"rounds_per_sync": ahead}, stats=True)
        od, _ = oracle.bfs(gg_, s)
        assert st["rounds"] == int(od[od != INF].max()) + 1
        lg = GG.bfs_log()
        assert st["rounds"] - 1 <= len(lg) <= st["rounds"]
        assert st["reached"] == int((od != INF).sum())
        deg = gg_.degrees()
        core = (od != INF) & ((deg >= 2) | (np.arange(gg_.n) == s))
        assert int(lg[:, 1].astype(np.int64).sum()) == int(core.sum())
        assert st["launches"] >= len(lg) + 1
        w, q, sw = gb.wbfs(GG, s, opts={"rounds_per_sync": ahead}, stats=True)
        ow, _ = oracle.wbfs(gg_, s)
        wl = GG.wbfs_log()
        assert len(wl) == sw["rounds"] + sw["pull_rounds"]
        assert len(np.unique(wl[:, 0])) == sw["rounds"]
        assert np.all(np.diff(wl[wl[:, 3] != 2, 0].astype(np.int64)) > 0)
        # buckets holding only stale entries are extracted too
        assert int(wl[:, 0].max()) >= int(ow[ow != 0xFFFFFFFF].max())


def test_unit_weights_equal_bfs(gb):
    g = gg.rmat(13, seed=4)
    g.weights = np.ones(g.m, dtype=np.int32)
    G = gb.Graph.from_csr(g)
    for s in gg.sources(g, 3, seed=3):
        d, p = run_bfs(gb, G, int(s))
        w, q = run_wbfs(gb, G, int(s))
        reach = d != 2**31 - 1
        assert np.array_equal(w[reach].astype(np.int64), d[reach])
        assert np.all(w[~reach] == 0xFFFFFFFF)
        assert np.array_equal(p, q)


def test_large_weights_and_isolated_source(gb):
    g = gg.rmat(12, seed=6)
    g.weights = gg.weights(g, 1000, seed=7)
    G = gb.Graph.from_csr(g)
    for s in gg.sources(g, 2, seed=3):
        assert_wbfs(gb, g, G, int(s), tag="w1000")
    iso = int(np.nonzero(g.degrees() == 0)[0][0])
    assert_bfs(gb, g, G, iso, tag="isolated")
    assert_wbfs(gb, g, G, iso, tag="isolated")


def test_erdos_renyi_and_torus(gb):
    for g in (gg.erdos_renyi(1 << 14, 32, seed=8), gg.torus3d(24)):
        g.weights = gg.weights(g, 24, seed=2)
        G = gb.Graph.from_csr(g)
        for s in gg.sources(g, 2, seed=3):
            assert_bfs(gb, g, G, int(s), tag=g.name)
            assert_wbfs(gb, g, G, int(s), tag=g.name)


def test_argument_errors(gb):
    g = gg.path(5)
    G = gb.Graph.from_csr(g)
    with pytest.raises(gb.GbgpuError) as e:
        gb.bfs(G, 5)
    assert e.value.status == gb.E_INVALID
    with pytest.raises(gb.GbgpuError) as e:
        gb.wbfs(G, 0)  # no weights
    assert e.value.status == gb.E_INVALID


def test_validation_rejects_malformed_graphs(gb):
    # asymmetric
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 1, 1]), np.array([1], dtype=np.int32))
    # unsorted list
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 2, 3, 4]), np.array([2, 1, 0, 0], dtype=np.int32))
    # self loop
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 1, 1]), np.array([0], dtype=np.int32))
    # bad offsets
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 2, 1]), np.array([1, 0], dtype=np.int32))
    # asymmetric weights
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 1, 2]), np.array([1, 0], dtype=np.int32),
                 np.array([3, 4], dtype=np.int32))
    # zero weight
    with pytest.raises(gb.GbgpuError):
        gb.Graph(np.array([0, 1, 2]), np.array([1, 0], dtype=np.int32),
                 np.array([0, 0], dtype=np.int32))


def test_back_to_back_calls_on_two_streams(gb, rmat16):
    """A BFS may return with empty launches still queued on its stream; a
    following call on the same graph from another stream must wait for them
    (outputs of both equal the oracle)."""
    g, G = rmat16
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    srcs = [int(x) for x in gg.sources(g, 6, seed=11)]
    outs = []
    for i, s in enumerate(srcs):
        st = s1 if i % 2 == 0 else s2
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        p = torch.empty(g.n, dtype=torch.int32, device="cuda")
        gb.bfs(G, s, dist=d, parent=p, stream=st, opts={"rounds_per_sync": 6})
        outs.append((s, d, p))
    torch.cuda.synchronize()
    for s, d, p in outs:
        od, op = oracle.bfs(g, s)
        assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op), s


@pytest.mark.parametrize("persistent", [1, -1])
def test_single_launch_rounds_identical(gb, persistent):
    """Every round in one cooperative launch (grid barriers between rounds)
    or one launch per round: the same outputs, equal to the oracle, on deep
    and shallow graphs, and over the whole range of grid sizes (one
    workgroup, a few per die, more than one per CU-die pair)."""
    for g in (gg.cycle(3001), gg.torus3d(24), gg.grid2d(70, 40), gg.rmat(14, seed=9),
              gg.path(2), gg.star(9)):
        G = gb.Graph.from_csr(g, with_weights=False)
        for i, s in enumerate(int(x) for x in gg.sources(g, 3, seed=11)):
            o = {"persistent": persistent, "grid": (0, 1, 37)[i]}
            d, p, st = gb.bfs(G, s, opts=o, stats=True)
            od, op = oracle.bfs(g, s)
            assert np.array_equal(d.cpu().numpy(), od), (g.name, s, o)
            assert np.array_equal(p.cpu().numpy(), op), (g.name, s, o)
            assert st["rounds"] == int(od[od != 2**31 - 1].max()) + 1
            if persistent == 1:
                assert st["launches"] == 1, (g.name, o, st)
        G.free()


def test_default_is_one_launch_per_round(gb):
    """Alone on the device the default keeps one launch per round, also on
    a graph a search has shown deep."""
    g = gg.cycle(501)
    G = gb.Graph.from_csr(g, with_weights=False)
    for s in (0, 7):
        d, p, st = gb.bfs(G, s, stats=True)
        assert st["launches"] > 1
        od, op = oracle.bfs(g, s)
        assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op)
    G.free()


def test_single_launch_many_workgroups_per_die(gb):
    """The single-launch form with hundreds of workgroups (dozens per die,
    so the die leaders' write-back and every workgroup's acquire carry the
    rounds), on a deep and on a shallow graph, and from an isolated source
    and from a degree-1 source."""
    for g in (gg.torus3d(48), gg.rmat(18, seed=4)):
        G = gb.Graph.from_csr(g, with_weights=False)
        deg = g.degrees()
        srcs = [int(x) for x in gg.sources(g, 2, seed=13)]
        if (deg == 0).any():
            srcs.append(int(np.nonzero(deg == 0)[0][0]))
        if (deg == 1).any():
            srcs.append(int(np.nonzero(deg == 1)[0][0]))
        for s in srcs:
            od, op = oracle.bfs(g, s)
            for grid in (256, 512):
                d, p, st = gb.bfs(G, s, opts={"persistent": 1, "grid": grid}, stats=True)
                assert np.array_equal(d.cpu().numpy(), od), (g.name, s, grid)
                assert np.array_equal(p.cpu().numpy(), op), (g.name, s, grid)
                assert st["launches"] == 1, (g.name, s, grid, st)
        G.free()


@pytest.mark.parametrize("force", [1, 2, 3])
def test_single_launch_forced_directions(gb, rmat16, force):
    """Push-only, pull-only and alternating rounds in one launch give the
    oracle's outputs, as they do one launch per round."""
    g, G = rmat16
    for s in gg.sources(g, 3, seed=17):
        d, p, st = gb.bfs(G, int(s), opts={"persistent": 1, "force_direction": force}, stats=True)
        od, op = oracle.bfs(g, int(s))
        assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op), (force, s)
        assert st["launches"] == 1
