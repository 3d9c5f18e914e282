"""The allocation-free BFS entry point (gbgpu_bfs_noalloc) through the C ABI:
its outputs equal gbgpu_bfs's element by element (and the oracle's) on two
calls in a row, the second on a smaller graph, then on the first graph
again; a graph larger than its static workspace is refused before any
launch, with the outputs untouched."""
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


def run_both(gb, G, s):
    d_ref, p_ref, st_ref = gb.bfs(G, s, stats=True)
    # outputs start as garbage: the entry point must write every entry
    d = torch.full((G.n,), 12345, dtype=torch.int32, device="cuda")
    p = torch.full((G.n,), -777, dtype=torch.int32, device="cuda")
    gb.bfs_noalloc(G, s, d, p)
    torch.cuda.synchronize()
    assert torch.equal(d, d_ref), "distances differ from gbgpu_bfs"
    assert torch.equal(p, p_ref), "parents differ from gbgpu_bfs"
    _, _, st = gb.bfs_noalloc(G, s, d, p, stats=True)
    for k in ("rounds", "reached", "push_rounds", "pull_rounds", "edges_examined"):
        assert st[k] == st_ref[k], (k, st[k], st_ref[k])
    return d.cpu().numpy(), p.cpu().numpy()


def test_noalloc_matches_bfs_on_two_calls_second_smaller(gb):
    big = gg.rmat(18, seed=1)
    small = gg.rmat(11, seed=4)
    Gb = gb.Graph.from_csr(big, with_weights=False)
    Gs = gb.Graph.from_csr(small, with_weights=False)
    sb = int(gg.sources(big, 1, seed=3)[0])
    ss = int(gg.sources(small, 1, seed=3)[0])
    d, p = run_both(gb, Gb, sb)
    od, op = oracle.bfs(big, sb)
    assert np.array_equal(d, od) and np.array_equal(p, op)
    d, p = run_both(gb, Gs, ss)
    od, op = oracle.bfs(small, ss)
    assert np.array_equal(d, od) and np.array_equal(p, op)
    # back to the larger graph, another source: nothing left over from the
    # smaller call changes the result
    sb2 = int(gg.sources(big, 2, seed=3)[1])
    run_both(gb, Gb, sb2)
    Gb.free()
    Gs.free()


def test_noalloc_deep_graph_and_isolated_source(gb):
    """Hundreds of rounds (the host checks progress every few launches) and
    a source without edges (the first round finds the frontier empty)."""
    g = gg.cycle(1000)
    G = gb.Graph.from_csr(g, with_weights=False)
    d, p = run_both(gb, G, 7)
    od, op = oracle.bfs(g, 7)
    assert np.array_equal(d, od) and np.array_equal(p, op)
    G.free()
    h = gg.from_edges(6, [(1, 2), (2, 3)])
    H = gb.Graph.from_csr(h, with_weights=False)
    d, p = run_both(gb, H, 0)
    assert d.tolist() == [0] + [2**31 - 1] * 5 and p.tolist() == [0] + [-1] * 5
    H.free()


def test_noalloc_refuses_a_graph_beyond_its_workspace(gb):
    n = 5_000_000  # needs about 82 MB of workspace; the array holds 64 MiB
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = 2
    off[0] = 0
    off[1] = 1
    nb = np.array([1, 0], dtype=np.int32)
    g = gg.CSR(n=n, offsets=off, nbrs=nb)
    G = gb.Graph.from_csr(g, validate=False, with_weights=False)
    d = torch.full((n,), 5, dtype=torch.int32, device="cuda")
    p = torch.full((n,), 6, dtype=torch.int32, device="cuda")
    with pytest.raises(gb.GbgpuError) as ei:
        gb.bfs_noalloc(G, 0, d, p)
    assert ei.value.status == gb.E_UNSUPPORTED
    torch.cuda.synchronize()
    assert bool((d == 5).all()) and bool((p == 6).all())
    # the regular entry point handles the same graph
    d2, p2 = gb.bfs(G, 0)
    assert d2[:3].tolist() == [0, 1, 2**31 - 1]
    G.free()
