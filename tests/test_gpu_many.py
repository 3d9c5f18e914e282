"""gbgpu_bfs_many: k single-source BFS back to back in one call, through the
C ABI, equal row by row to the oracle (and so to k gbgpu_bfs calls)."""
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


@pytest.mark.parametrize("make", [lambda: gg.rmat(14, seed=2), lambda: gg.torus3d(12),
                                  lambda: gg.rmat(12, edge_factor=2, seed=4)])
def test_rows_match_the_oracle(gb, make):
    g = make()
    G = gb.Graph.from_csr(g)
    srcs = [int(x) for x in gg.sources(g, 9, seed=5)] + [0]   # vertex 0 may be isolated
    d, p, st = gb.bfs_many(G, srcs, stats=True)
    d = d.cpu().numpy()
    p = p.cpu().numpy()
    reached = 0
    for i, s in enumerate(srcs):
        ed, ep = oracle.bfs(g, s)
        assert np.array_equal(d[i], ed) and np.array_equal(p[i], ep), f"row {i} src {s}"
        reached += int((ed != oracle.BFS_INF).sum())
    assert st["reached"] == reached
    # one shared output: it ends holding the last search
    d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    gb.bfs_many(G, srcs[::-1], dist=d1, parent=p1, row_stride=0, opts={"force_direction": 2})
    ed, ep = oracle.bfs(g, srcs[0])
    assert np.array_equal(d1.cpu().numpy(), ed) and np.array_equal(p1.cpu().numpy(), ep)
    G.free()


def test_argument_errors(gb):
    g = gg.rmat(8, seed=1)
    G = gb.Graph.from_csr(g)
    with pytest.raises(gb.GbgpuError):
        gb.bfs_many(G, [0, g.n])
    with pytest.raises(gb.GbgpuError):
        gb.bfs_many(G, [])
    d = torch.empty(4 * g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(gb.GbgpuError):
        gb.bfs_many(G, [0, 1], dist=d, parent=d.clone(), row_stride=g.n - 1)
    G.free()
