"""GPU parity at the benchmark's full sizes, in its launch configuration
(default options, plus the tuned settings stored for each graph):

* RMAT scale 24: BFS from the first two timed sources and weighted BFS
  (w < 24) from the first, element by element against the oracle; two rows
  of a 64-source batch against the oracle;
* 256^3 torus: BFS, and 64 sources batched (rows 0, 31, 63), against the
  closed form of distances and min-ID parents,
  weighted BFS (w < 24) against the definition-level checks;
* general-weight SSSP and widest path (w < 24) from the first timed source:
  RMAT-24 against the oracle's Bellman-Ford and widest path, the torus
  against the oracle's Dial distances (equal to Bellman-Ford's on
  positive weights; its own passes would number in the hundreds there) and
  widest path;
* single-source betweenness from the first timed source, RMAT-24 and torus,
  against the oracle within the tolerance of test_gpu_bc.py;
* low-diameter decomposition (beta 0.2, the seed the benchmark uses) and
  connectivity, RMAT-24 and torus, element by element against the oracle;
* compressed adjacency: RMAT-24 decoded back exactly, and BFS over the
  compressed lists from the first two timed sources against the oracle;
  torus 256^3 against the closed form.
"""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from checks import check_wbfs
from test_oracle import torus_closed_form

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TUNED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1805_05208_amd", "tuned.json")


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_05208_amd as m
    m.lib()
    return m


def tuned(sig_prefix, kind):
    with open(TUNED) as f:
        db = json.load(f)
    for sig, kinds in db.items():
        if sig.startswith(sig_prefix) and kind in kinds:
            return kinds[kind]["opts"]
    return None


@pytest.fixture(scope="module")
def rmat24(gb):
    g = gg.rmat(24, seed=1)
    w = gg.weights(g, 24, seed=2)
    G = gb.Graph(g.offsets, g.nbrs, w, validate=False)
    yield g, w, G
    G.free()


def assert_same(d, p, od, op, tag):
    d = np.asarray(d)
    p = np.asarray(p)
    bad = np.nonzero((d != od) | (p != op))[0]
    assert bad.size == 0, (f"{tag}: {bad.size} mismatches, first v={bad[0]}: gpu "
                           f"({d[bad[0]]},{p[bad[0]]}) oracle ({od[bad[0]]},{op[bad[0]]})")


def test_rmat24_bfs(gb, rmat24):
    g, _, G = rmat24
    opts = tuned(f"n{g.n}-m{g.m}-", "bfs")
    for s in [int(x) for x in gg.sources(g, 16, seed=3)[:2]]:
        d, p = gb.bfs(G, s, opts=opts)
        od, op = oracle.bfs(g, s)
        assert_same(d.cpu().numpy(), p.cpu().numpy(), od, op, f"rmat24 bfs src={s}")


def test_rmat24_wbfs(gb, rmat24):
    g, w, G = rmat24
    s = int(gg.sources(g, 16, seed=3)[0])
    d, p = gb.wbfs(G, s, opts=tuned(f"n{g.n}-m{g.m}-", "wbfs"))
    od, op = oracle.wbfs(g, s, weights=w)
    assert_same(gb.as_u32(d), p.cpu().numpy(), od, op, f"rmat24 wbfs src={s}")


def test_rmat24_batched_rows(gb, rmat24):
    g, _, G = rmat24
    s64 = [int(x) for x in gg.sources(g, 64, seed=3)]
    D, P = gb.bfs_multi(G, s64)
    for i in (5, 40):
        od, op = oracle.bfs(g, s64[i])
        assert_same(D[i].cpu().numpy(), P[i].cpu().numpy(), od, op, f"rmat24 batch row {i}")
    del D, P
    torch.cuda.empty_cache()


def test_torus256(gb):
    g = gg.torus3d(256).with_weights(24, seed=2)
    G = gb.Graph.from_csr(g, validate=False)
    s = int(gg.sources(g, 1, seed=3)[0])
    prefix = f"n{g.n}-m{g.m}-"
    d, p = gb.bfs(G, s, opts=tuned(prefix, "bfs"))
    ed, ep = torus_closed_form(256, s)
    assert_same(d.cpu().numpy(), p.cpu().numpy(), ed, ep, "torus256 bfs")
    wd, wp = gb.wbfs(G, s, opts=tuned(prefix, "wbfs"))
    check_wbfs(g, s, gb.as_u32(wd), wp.cpu().numpy())
    G.free()


def test_torus256_batched_rows(gb):
    """64 sources on the 256^3 torus in one gbgpu_bfs_multi call, as the
    benchmark times it: the graph is known to be 385 levels deep, so the pair
    entries are 8 bytes from the start; rows 0, 31 and 63 against the closed
    form."""
    g = gg.torus3d(256)
    G = gb.Graph.from_csr(g, validate=False, with_weights=False)
    srcs = [int(x) for x in gg.sources(g, 64, seed=3)]
    _, _, st = gb.bfs(G, srcs[0], stats=True)
    assert st["rounds"] > 254
    D, P = gb.bfs_multi(G, srcs)
    for i in (0, 31, 63):
        ed, ep = torus_closed_form(256, srcs[i])
        assert_same(D[i].cpu().numpy(), P[i].cpu().numpy(), ed, ep, f"torus256 batched row {i}")
    del D, P
    G.free()
    torch.cuda.empty_cache()


def test_rmat24_bellman_ford_and_widest_path(gb, rmat24):
    g, w, G = rmat24
    s = int(gg.sources(g, 16, seed=3)[0])
    d = gb.bellman_ford(G, s).cpu().numpy()
    ref = oracle.bellman_ford(g, s, w)
    bad = np.nonzero(d != ref)[0]
    assert bad.size == 0, f"bellman-ford: {bad.size} mismatches, first v={bad[0]}"
    wd = gb.as_u32(gb.widest_path(G, s))
    wref = oracle.widest_path(g, s, w)
    bad = np.nonzero(wd != wref)[0]
    assert bad.size == 0, f"widest path: {bad.size} mismatches, first v={bad[0]}"


def test_torus256_bellman_ford_and_widest_path(gb):
    g = gg.torus3d(256).with_weights(24, seed=2)
    G = gb.Graph.from_csr(g, validate=False)
    s = int(gg.sources(g, 1, seed=3)[0])
    d = gb.bellman_ford(G, s).cpu().numpy()
    dd, _ = oracle.wbfs(g, s)
    exp = np.where(dd == oracle.WBFS_INF, np.int64(2**63 - 1), dd.astype(np.int64))
    assert np.array_equal(d, exp)
    wd = gb.as_u32(gb.widest_path(G, s))
    assert np.array_equal(wd, oracle.widest_path(g, s))
    G.free()


@pytest.mark.parametrize("which", ["rmat24", "torus256"])
def test_betweenness(gb, which, request):
    from test_gpu_bc import assert_close, oracle_levels, rtol_for
    if which == "rmat24":
        g, _, G = request.getfixturevalue("rmat24")
        s = int(gg.sources(g, 16, seed=3)[0])
        own = False
    else:
        g = gg.torus3d(256)
        G = gb.Graph.from_csr(g, validate=False, with_weights=False)
        s = int(gg.sources(g, 1, seed=3)[0])
        own = True
    dep = gb.betweenness(G, s)
    exp = oracle.betweenness(g, s)
    assert_close(dep.cpu().numpy(), exp, rtol_for(g, oracle_levels(g, s)), f"{which} src={s}")
    if own:
        G.free()


@pytest.mark.parametrize("which", ["rmat24", "torus256"])
def test_ldd_and_connectivity(gb, which, request):
    if which == "rmat24":
        g, _, G = request.getfixturevalue("rmat24")
        own = False
    else:
        g = gg.torus3d(256)
        G = gb.Graph.from_csr(g, validate=False, with_weights=False)
        own = True
    cl = gb.ldd(G, 0.2, 1).cpu().numpy()
    exp = oracle.ldd(g, 0.2, 1)
    bad = np.nonzero(cl != exp)[0]
    assert bad.size == 0, f"{which} LDD: {bad.size} differ, first v={bad[0]}"
    lab = gb.connectivity(G, 0.2, 1).cpu().numpy()
    exp = oracle.components(g)
    bad = np.nonzero(lab != exp)[0]
    assert bad.size == 0, f"{which} connectivity: {bad.size} differ, first v={bad[0]}"
    if own:
        G.free()


def test_rmat24_compressed(gb, rmat24):
    g, _, G = rmat24
    gb.compress(G)
    assert np.array_equal(gb.decompress(G).cpu().numpy(), g.nbrs)
    for s in [int(x) for x in gg.sources(g, 16, seed=3)[:2]]:
        d, p = gb.bfs_compressed(G, s)
        od, op = oracle.bfs(g, s)
        assert_same(d.cpu().numpy(), p.cpu().numpy(), od, op, f"rmat24 compressed src={s}")


def test_torus256_compressed(gb):
    g = gg.torus3d(256)
    G = gb.Graph.from_csr(g, validate=False, with_weights=False)
    gb.compress(G)
    s = int(gg.sources(g, 1, seed=3)[0])
    d, p = gb.bfs_compressed(G, s)
    ed, ep = torus_closed_form(256, s)
    assert_same(d.cpu().numpy(), p.cpu().numpy(), ed, ep, "torus256 compressed")
    G.free()
