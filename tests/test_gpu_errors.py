"""Weight-dependent limits of the weighted BFS, through the C ABI: the
library learns the largest weight on the device at load time, and a
weighted BFS (or a served weighted query) on a graph beyond its limits is
refused before any traversal launch, with the outputs left untouched:

* E_UNSUPPORTED when the largest weight exceeds 2047 (the bucket ring holds
  at most 2 * 2047 + 1 distances);
* E_OVERFLOW when max_weight * n >= 2^32 - 2 (a tentative distance could
  exceed the 32-bit range);
* BFS, Bellman-Ford and widest path on the same graphs still run.
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


def path_with_weights(n, heavy):
    """A path on the first 3 vertices (weights 1 and `heavy`), every other
    vertex isolated."""
    off = np.zeros(n + 1, dtype=np.int64)
    off[1] = 1
    off[2] = 3
    off[3:] = 4
    nbrs = np.array([1, 0, 2, 1], dtype=np.int32)
    w = np.array([1, 1, heavy, heavy], dtype=np.int32)
    return gg.CSR(n=n, offsets=off, nbrs=nbrs, weights=w)


def untouched(gb, g, call):
    d = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    p = torch.full((g.n,), 9, dtype=torch.int32, device="cuda")
    with pytest.raises(gb.GbgpuError) as e:
        call(d, p)
    torch.cuda.synchronize()
    assert bool((d == 7).all()) and bool((p == 9).all()), "outputs written on an error"
    return e.value.status


def test_weight_above_2047_is_unsupported(gb):
    g = path_with_weights(8, 2048)
    G = gb.Graph.from_csr(g)
    assert untouched(gb, g, lambda d, p: gb.wbfs(G, 0, dist=d, parent=p)) == gb.E_UNSUPPORTED
    sv = gb.Server(arena_bytes=64 << 20, max_inflight=1)
    gid = sv.add_graph(G)
    assert untouched(gb, g, lambda d, p: sv.submit(gid, gb.QUERY_WBFS, 0, d, p)) == \
        gb.E_UNSUPPORTED
    sv.close()
    # the other traversals accept the graph
    d, p = gb.bfs(G, 0)
    od, op = oracle.bfs(g, 0)
    assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op)
    assert gb.bellman_ford(G, 0).cpu().tolist()[:3] == [0, 1, 2049]
    assert gb.as_u32(gb.widest_path(G, 0))[:3].tolist() == [0xFFFFFFFF, 1, 1]
    G.free()
    # 2047 is accepted
    h = path_with_weights(8, 2047)
    H = gb.Graph.from_csr(h)
    d, p = gb.wbfs(H, 0)
    assert gb.as_u32(d)[:3].tolist() == [0, 1, 2048] and p.cpu().tolist()[:3] == [0, 0, 1]
    H.free()


def test_distance_range_overflow(gb):
    # 2047 * n >= 2^32 - 2 once n >= 2 098 177
    n = 2_098_177
    g = path_with_weights(n, 2047)
    G = gb.Graph.from_csr(g, validate=False)
    assert untouched(gb, g, lambda d, p: gb.wbfs(G, 0, dist=d, parent=p)) == gb.E_OVERFLOW
    sv = gb.Server(arena_bytes=1 << 30, max_inflight=1)
    gid = sv.add_graph(G)
    assert untouched(gb, g, lambda d, p: sv.submit(gid, gb.QUERY_WBFS, 0, d, p)) == \
        gb.E_OVERFLOW
    sv.close()
    G.free()
    # one vertex fewer fits
    h = path_with_weights(n - 1, 2047)
    H = gb.Graph.from_csr(h, validate=False)
    d, p = gb.wbfs(H, 2)
    assert gb.as_u32(d)[:3].tolist() == [2048, 2047, 0]
    H.free()
