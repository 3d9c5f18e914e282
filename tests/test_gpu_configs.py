"""GPU parity of every benchmark configuration at its own size, in the
launch configuration the benchmark times, element by element against the
oracle (run on several host threads: the oracle is single-threaded C and
each call is independent):

1. RMAT scale 16: BFS from each of 16 seeded sources.
2. RMAT scale 24: BFS from all 16 timed sources through one gbgpu_bfs_many
   call (the benchmark's step) with the stored tuned options.
3. Weighted BFS (w in [1, 24)): RMAT scale 24 from the first 4 timed
   sources; 256^3 torus from 4 seeded sources (oracle's Dial search, besides
   the closed form of BFS on the torus checked elsewhere).
4. Batched BFS: all 64 rows of the 64-source RMAT-24 batch; all 256 rows of
   the uneven batch over RMAT scales 12..18 and 20 (32 queries per graph).
5. Serving: one BFS and one weighted BFS on each of the six resident graphs
   (RMAT 18/22/24/26, 256^3 torus, Erdos-Renyi 2^23 of average degree 32,
   weights in [1, log2 n)) submitted together, each equal to the standalone
   call and to the oracle.

These are the slowest GPU tests (graph generation and oracle runs on the
host dominate); they are marked slow as well as gpu.
"""
import concurrent.futures as cf
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

TUNED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1805_05208_amd", "tuned.json")
# oracle threads: one process may use up to 16 host cores
WORKERS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_05208_amd as m
    m.lib()
    return m


def tuned(g, kind):
    with open(TUNED) as f:
        db = json.load(f)
    prefix = f"n{g.n}-m{g.m}-"
    for sig, kinds in db.items():
        if sig.startswith(prefix) and kind in kinds:
            return kinds[kind]["opts"]
    return None


def oracle_map(fn, calls):
    """fn(*args) for every args tuple in calls, on WORKERS host threads (the
    oracle's ctypes calls release the interpreter lock)."""
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(lambda a: fn(*a), calls))


def assert_same(d, p, od, op, tag):
    d = np.asarray(d)
    p = np.asarray(p)
    bad = np.nonzero((d != od) | (p != op))[0]
    assert bad.size == 0, (f"{tag}: {bad.size} mismatches, first v={bad[0]}: gpu "
                           f"({d[bad[0]]},{p[bad[0]]}) oracle ({od[bad[0]]},{op[bad[0]]})")


@pytest.fixture(scope="module")
def rmat24(gb):
    g = gg.rmat(24, seed=1)
    w = gg.weights(g, 24, seed=2)
    G = gb.Graph(g.offsets, g.nbrs, w, validate=False)
    yield g, w, G
    G.free()
    torch.cuda.empty_cache()


def test_config1_rmat16_bfs(gb):
    g = gg.rmat(16, seed=1)
    G = gb.Graph.from_csr(g, with_weights=False)
    srcs = [int(s) for s in gg.sources(g, 16, seed=3)]
    exp = oracle_map(oracle.bfs, [(g, s) for s in srcs])
    # the library defaults and the tuned options the benchmark times
    for opts in (None, tuned(g, "bfs")):
        for s, (od, op) in zip(srcs, exp):
            d, p = gb.bfs(G, s, opts=opts)
            assert_same(d.cpu().numpy(), p.cpu().numpy(), od, op, f"rmat16 src={s} opts={opts}")
    G.free()


def test_config2_rmat24_all_timed_sources(gb, rmat24):
    g, _, G = rmat24
    srcs = [int(s) for s in gg.sources(g, 16, seed=3)]
    D, P = gb.bfs_many(G, srcs, opts=tuned(g, "bfs"))
    D = D.cpu().numpy()
    P = P.cpu().numpy()
    exp = oracle_map(oracle.bfs, [(g, s) for s in srcs])
    for i, (s, (od, op)) in enumerate(zip(srcs, exp)):
        assert_same(D[i], P[i], od, op, f"rmat24 timed source {i} ({s})")


def test_config3_rmat24_wbfs_four_sources(gb, rmat24):
    g, w, G = rmat24
    srcs = [int(s) for s in gg.sources(g, 16, seed=3)[:4]]
    opts = tuned(g, "wbfs")
    got = []
    for s in srcs:
        d, p = gb.wbfs(G, s, opts=opts)
        got.append((gb.as_u32(d), p.cpu().numpy()))
    exp = oracle_map(oracle.wbfs, [(g, s, w) for s in srcs])
    for s, (d, p), (od, op) in zip(srcs, got, exp):
        assert_same(d, p, od, op, f"rmat24 wbfs src={s}")


def test_config3_torus256_wbfs_four_sources(gb):
    g = gg.torus3d(256).with_weights(24, seed=2)
    G = gb.Graph.from_csr(g, validate=False)
    srcs = [int(s) for s in gg.sources(g, 4, seed=3)]
    opts = tuned(g, "wbfs")
    got = []
    for s in srcs:
        d, p = gb.wbfs(G, s, opts=opts)
        got.append((gb.as_u32(d), p.cpu().numpy()))
    exp = oracle_map(oracle.wbfs, [(g, s) for s in srcs])
    for s, (d, p), (od, op) in zip(srcs, got, exp):
        assert_same(d, p, od, op, f"torus256 wbfs src={s}")
    G.free()


def test_config4_rmat24_all_64_batch_rows(gb, rmat24):
    g, _, G = rmat24
    s64 = [int(x) for x in gg.sources(g, 64, seed=3)]
    D, P = gb.bfs_multi(G, s64)
    D = D.cpu().numpy()
    P = P.cpu().numpy()
    torch.cuda.empty_cache()
    exp = oracle_map(oracle.bfs, [(g, s) for s in s64])
    for i, (s, (od, op)) in enumerate(zip(s64, exp)):
        assert_same(D[i], P[i], od, op, f"rmat24 batch row {i} ({s})")


def test_config4_uneven_batch_all_256_rows(gb):
    scales = [12, 13, 14, 15, 16, 17, 18, 20]
    graphs = [gg.rmat(sc, seed=1) for sc in scales]
    Gs = [gb.Graph.from_csr(h, validate=False, with_weights=False) for h in graphs]
    qi, qs = [], []
    for i, h in enumerate(graphs):
        for s in gg.sources(h, 32, seed=3):
            qi.append(i)
            qs.append(int(s))
    assert len(qs) == 256
    dists, parents = gb.bfs_batch([Gs[i] for i in qi], qs)
    exp = oracle_map(oracle.bfs, [(graphs[i], s) for i, s in zip(qi, qs)])
    for q, (od, op) in enumerate(exp):
        assert_same(dists[q].cpu().numpy(), parents[q].cpu().numpy(), od, op,
                    f"uneven query {q} (rmat{scales[qi[q]]} src={qs[q]})")
    for G_ in Gs:
        G_.free()


def serving_graphs():
    """The six resident graphs of the serving configuration, weights in
    [1, log2 n)."""
    return [("rmat18", lambda: gg.rmat(18, seed=1), 18),
            ("rmat22", lambda: gg.rmat(22, seed=1), 22),
            ("rmat24", lambda: gg.rmat(24, seed=1), 24),
            ("rmat26", lambda: gg.rmat(26, seed=1), 26),
            ("torus256", lambda: gg.torus3d(256), 24),
            ("er23", lambda: gg.erdos_renyi(1 << 23, 32, seed=1), 23)]


def test_config5_served_queries_on_every_resident_graph(gb):
    """One BFS and one weighted BFS per resident graph, all submitted before
    any is collected (so they share the device), each equal to the
    standalone library call and to the oracle."""
    graphs = []
    for name, make, W in serving_graphs():
        h = make().with_weights(W, seed=2)
        graphs.append((name, h, gb.Graph.from_csr(h, validate=False)))
    sv = gb.Server(arena_bytes=96 << 30, max_inflight=8)
    ids = [sv.add_graph(G) for _, _, G in graphs]
    jobs = []
    for gi, (name, h, _G) in enumerate(graphs):
        s = int(gg.sources(h, 1, seed=3)[0])
        for kind in (0, 1):
            d = torch.empty(h.n, dtype=torch.int32, device="cuda")
            p = torch.empty(h.n, dtype=torch.int32, device="cuda")
            jobs.append((gi, kind, s, d, p, sv.submit(ids[gi], kind, s, d, p)))
    sv.drain()
    for gi, kind, s, d, p, t in jobs:
        r = sv.poll(t)
        assert r is not None and r["status"] == 0, (graphs[gi][0], kind, r)
    sv.close()
    # standalone calls on the same graphs and sources
    served = []
    for gi, kind, s, d, p, _t in jobs:
        G = graphs[gi][2]
        sd, sp = (gb.bfs if kind == 0 else gb.wbfs)(G, s)
        assert torch.equal(sd, d) and torch.equal(sp, p), \
            f"{graphs[gi][0]} kind {kind}: served result differs from the standalone call"
        served.append((d.cpu().numpy(), p.cpu().numpy()))
        del sd, sp
    for _, _, G in graphs:
        G.free()
    torch.cuda.empty_cache()

    def ref(gi, kind, s):
        h = graphs[gi][1]
        return oracle.bfs(h, s) if kind == 0 else oracle.wbfs(h, s)

    exp = oracle_map(ref, [(gi, kind, s) for gi, kind, s, _d, _p, _t in jobs])
    for (gi, kind, s, _d, _p, _t), (d, p), (od, op) in zip(jobs, served, exp):
        if kind == 1:
            d = d.view(np.uint32)
        assert_same(d, p, od, op, f"served {graphs[gi][0]} {'bfs' if kind == 0 else 'wbfs'} src={s}")
