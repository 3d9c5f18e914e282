"""GPU tests of the query server: every result equals the oracle and the
standalone call, alone and in a mix; admission errors are reported."""
import time

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


@pytest.fixture(scope="module")
def graphs(gb):
    gs = [gg.rmat(13, seed=51).with_weights(13, seed=2),
          gg.torus3d(12).with_weights(10, seed=3),
          gg.erdos_renyi(1 << 12, 16, seed=52).with_weights(12, seed=4)]
    return gs, [gb.Graph.from_csr(g) for g in gs]


def wait(sv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = sv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.0005)
    return out


def test_server_mixed_stream_matches_oracle(gb, graphs):
    gs, Gs = graphs
    sv = gb.Server(arena_bytes=256 << 20, max_inflight=4)
    ids = [sv.add_graph(G) for G in Gs]
    rng = np.random.default_rng(1)
    jobs = []
    for i in range(60):
        gi = int(rng.integers(0, 3))
        kind = int(rng.integers(0, 2))
        src = int(gg.sources(gs[gi], 20, seed=60 + gi)[int(rng.integers(0, 20))])
        d = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        p = torch.empty(gs[gi].n, dtype=torch.int32, device="cuda")
        t = sv.submit(ids[gi], kind, src, d, p)
        jobs.append((t, gi, kind, src, d, p))
    res = wait(sv, [j[0] for j in jobs])
    for t, gi, kind, src, d, p in jobs:
        assert res[t]["status"] == gb.OK
        assert res[t]["t_arrive_ns"] <= res[t]["t_start_ns"] <= res[t]["t_done_ns"]
        if kind == gb.QUERY_BFS:
            od, op = oracle.bfs(gs[gi], src)
            assert np.array_equal(d.cpu().numpy(), od)
        else:
            od, op = oracle.wbfs(gs[gi], src)
            assert np.array_equal(gb.as_u32(d), od)
        assert np.array_equal(p.cpu().numpy(), op)
        # the standalone call gives the same result
        sd, sp = (gb.bfs if kind == gb.QUERY_BFS else gb.wbfs)(Gs[gi], src)
        assert torch.equal(sd, d) and torch.equal(sp, p)
    sv.close()


def test_server_small_arena_serialises_and_overflow_requeue(gb, graphs):
    gs, Gs = graphs
    g, G = gs[0], Gs[0]
    need = G.footprint(gb.QUERY_WBFS)
    # room for exactly one default weighted query: admission must serialise,
    # and a tiny bucket capacity forces re-queues with larger buckets
    sv = gb.Server(arena_bytes=need * 3, max_inflight=3, opts={"bucket_capacity": 64})
    gid = sv.add_graph(G)
    srcs = gg.sources(g, 6, seed=9)
    outs = []
    for s in srcs:
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        p = torch.empty(g.n, dtype=torch.int32, device="cuda")
        outs.append((sv.submit(gid, gb.QUERY_WBFS, int(s), d, p), int(s), d, p))
    res = wait(sv, [o[0] for o in outs])
    for t, s, d, p in outs:
        od, op = oracle.wbfs(g, s)
        assert res[t]["status"] == gb.OK
        assert np.array_equal(gb.as_u32(d), od) and np.array_equal(p.cpu().numpy(), op)
    sv.close()


def test_server_learned_capacity_and_batching_rule(gb, graphs):
    """A weighted query after one that had to grow its buckets starts with
    the grown capacity; BFS queries on a graph no search has measured run one
    at a time, later ones on the (shallow, small) graph bit-packed.  Every
    result equals the oracle either way."""
    gs, _ = graphs
    g = gs[2]
    G = gb.Graph.from_csr(g)          # fresh handle: depth not yet known
    sv = gb.Server(arena_bytes=1 << 30, max_inflight=4, opts={"bucket_capacity": 64})
    gid = sv.add_graph(G)
    srcs = [int(x) for x in gg.sources(g, 12, seed=33)]

    def run(kind, ss):
        outs = []
        for s in ss:
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            p = torch.empty(g.n, dtype=torch.int32, device="cuda")
            outs.append((sv.submit(gid, kind, s, d, p), s, d, p))
        res = wait(sv, [o[0] for o in outs])
        for t, s, d, p in outs:
            assert res[t]["status"] == gb.OK
            od, op = (oracle.bfs if kind == gb.QUERY_BFS else oracle.wbfs)(g, s)
            dd = d.cpu().numpy() if kind == gb.QUERY_BFS else gb.as_u32(d)
            assert np.array_equal(dd, od) and np.array_equal(p.cpu().numpy(), op), (kind, s)
        return [res[o[0]] for o in outs]

    first = run(gb.QUERY_WBFS, srcs[:1])      # overflows 64 and grows
    assert first[0]["retries"] >= 1 and first[0]["batch"] == 1
    # the same source again starts from the capacity it grew to: no rerun
    again = run(gb.QUERY_WBFS, srcs[:1] * 2)
    assert [r["retries"] for r in again] == [0, 0]
    run(gb.QUERY_WBFS, srcs[1:4])
    alone = run(gb.QUERY_BFS, srcs[:1])       # depth unknown: alone
    assert alone[0]["batch"] == 1
    sv.close()
    # shallow and small, the graph's BFS queries are now packed: they arrive
    # while the one worker of a second server is busy with a long weighted
    # query (a 40^3 torus, about 120 buckets), so they wait together
    t = gg.torus3d(40).with_weights(8, seed=1)
    T = gb.Graph.from_csr(t)
    sv = gb.Server(arena_bytes=1 << 30, max_inflight=1)
    gid, tid = sv.add_graph(G), sv.add_graph(T)
    tb = [torch.empty(t.n, dtype=torch.int32, device="cuda") for _ in range(2)]
    outs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"),
             torch.empty(g.n, dtype=torch.int32, device="cuda")) for _ in srcs]
    torch.cuda.synchronize()
    blocker = sv.submit(tid, gb.QUERY_WBFS, 0, tb[0], tb[1])
    tickets = [sv.submit(gid, gb.QUERY_BFS, s, d, p) for s, (d, p) in zip(srcs, outs)]
    res = wait(sv, [blocker] + tickets)
    assert res[blocker]["status"] == gb.OK
    packed = [res[x] for x in tickets]
    for r, s, (d, p) in zip(packed, srcs, outs):
        assert r["status"] == gb.OK
        od, op = oracle.bfs(g, s)
        assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op), s
    assert max(r["batch"] for r in packed) > 1
    # the queries that started a packed run share its start time and report
    # its size: they plus the queries that joined it at a round boundary
    # (join_round > 0, each with the time it joined as its start)
    by_start = {}
    joined = [r for r in packed if r["join_round"] > 0]
    for r in packed:
        if r["join_round"] == 0:
            by_start.setdefault(r["t_start_ns"], []).append(r["batch"])
    extra = 0
    for bs in by_start.values():
        assert len(set(bs)) == 1 and bs[0] >= len(bs), by_start
        extra += bs[0] - len(bs)
    assert extra == len(joined), (by_start, joined)
    sizes = {bs[0] for bs in by_start.values()}
    assert all(r["batch"] in sizes for r in joined), (by_start, joined)
    sv.close()
    G.free()
    T.free()


def test_server_errors(gb, graphs):
    gs, Gs = graphs
    sv = gb.Server(arena_bytes=1 << 16, max_inflight=1, opts={"max_pending": 2})
    gid = sv.add_graph(Gs[0])
    d = torch.empty(gs[0].n, dtype=torch.int32, device="cuda")
    p = torch.empty(gs[0].n, dtype=torch.int32, device="cuda")
    with pytest.raises(gb.GbgpuError) as e:  # footprint larger than the arena
        sv.submit(gid, gb.QUERY_BFS, 0, d, p)
    assert e.value.status == gb.E_NOMEM
    with pytest.raises(gb.GbgpuError) as e:
        sv.submit(gid + 5, gb.QUERY_BFS, 0, d, p)
    assert e.value.status == gb.E_INVALID
    with pytest.raises(gb.GbgpuError) as e:
        sv.poll(12345)
    assert e.value.status == gb.E_NOTFOUND
    sv.close()
    # a full pending queue reports E_AGAIN (arena too small to start anything
    # is avoided by using a single worker blocked on a large arena request)
    sv = gb.Server(arena_bytes=Gs[0].footprint(gb.QUERY_BFS) + 4096, max_inflight=1,
                   opts={"max_pending": 2})
    gid = sv.add_graph(Gs[0])
    tickets, again = [], 0
    for i in range(50):
        t = sv.try_submit(gid, gb.QUERY_BFS, int(gg.sources(gs[0], 1, seed=i + 1)[0]), d, p)
        if t is None:
            again += 1
        else:
            tickets.append(t)
    assert again > 0
    wait(sv, tickets)
    sv.close()


def test_arrivals_join_a_running_packed_group(gb):
    """BFS arrivals on a graph whose packed group is running join it at a
    round boundary (join_round > 0, one group start time for the starters).
    A slow weighted query first holds the only worker, so two BFS queries on
    a shallow 120-cycle (depth 61, known from a first search) start together
    as a group with room for 64; ten more arrive while it runs.  Every result
    equals the oracle whatever the timing; at least one of five attempts
    must show a join."""
    ring = gg.cycle(120)
    R = gb.Graph.from_csr(ring, with_weights=False)
    gb.bfs(R, 0)  # the graph's depth becomes known: packable
    big = gg.rmat(16, seed=3).with_weights(16, seed=2)
    B = gb.Graph.from_csr(big)
    sv = gb.Server(arena_bytes=1 << 30, max_inflight=1)
    rid, bid = sv.add_graph(R), sv.add_graph(B)
    joined_any = False
    for attempt in range(5):
        outs = []

        def submit(gid, kind, src, n):
            d = torch.empty(n, dtype=torch.int32, device="cuda")
            p = torch.empty(n, dtype=torch.int32, device="cuda")
            outs.append((sv.submit(gid, kind, src, d, p), gid, kind, src, d, p))
            return outs[-1][0]

        blocker = submit(bid, gb.QUERY_WBFS, int(gg.sources(big, 1, seed=attempt + 1)[0]), big.n)
        for s in (3 + attempt, 60):
            submit(rid, gb.QUERY_BFS, s, ring.n)
        while sv.poll(blocker) is None:
            time.sleep(0.0001)
        for s in range(10):
            submit(rid, gb.QUERY_BFS, (11 * s + attempt) % ring.n, ring.n)
        res = wait(sv, [o[0] for o in outs[1:]])
        for t, gid, kind, s, d, p in outs[1:]:
            assert res[t]["status"] == gb.OK
            od, op = oracle.bfs(ring, s)
            assert np.array_equal(d.cpu().numpy(), od) and np.array_equal(p.cpu().numpy(), op), s
        joins = [res[o[0]]["join_round"] for o in outs[1:]]
        if any(j > 0 for j in joins):
            joined_any = True
            # the queries that joined report the group's size and later start
            starters = [res[o[0]] for o in outs[1:3]]
            late = [res[o[0]] for o in outs[3:] if res[o[0]]["join_round"] > 0]
            assert all(r["batch"] >= 3 for r in starters + late)
            assert all(r["t_start_ns"] > starters[0]["t_start_ns"] for r in late)
            break
    sv.close()
    R.free()
    B.free()
    assert joined_any, "no arrival joined a running group in five attempts"


@pytest.mark.skip(reason="the server's single-launch BFS is not run: a serving benchmark "
                         "process that used it (deep graphs, 128 workgroups) ended in a "
                         "segmentation fault at exit after every result had been verified; "
                         "the cause is not found, so the path stays off")
def test_bfs_served_in_one_launch(gb):
    """A server created with persistent = 1 runs its BFS queries as one
    launch each (every round behind grid barriers), beside queries on
    other graphs; with the default, one launch per round.  Every result
    equals the oracle."""
    deep, shallow = gg.grid2d(300, 20), gg.rmat(12, seed=8)
    Gd = gb.Graph.from_csr(deep, with_weights=False)
    Gs = gb.Graph.from_csr(shallow, with_weights=False)
    for opts, single in (({"persistent": 1}, True), (None, False)):
        sv = gb.Server(arena_bytes=64 << 20, max_inflight=4, opts=opts)
        gd, gs_ = sv.add_graph(Gd), sv.add_graph(Gs)
        ss = [int(x) for x in gg.sources(shallow, 4, seed=3)]
        out = []
        for gid, g, s in ((gd, deep, 150), (gs_, shallow, ss[0]), (gd, deep, 4321),
                          (gs_, shallow, ss[1]), (gd, deep, 5999)):
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            p = torch.empty(g.n, dtype=torch.int32, device="cuda")
            out.append((sv.submit(gid, gb.QUERY_BFS, s, d, p), g, s, d, p))
        res = wait(sv, [o[0] for o in out])
        for t, g, s, d, p in out:
            assert res[t]["status"] == gb.OK
            od, op = oracle.bfs(g, s)
            assert np.array_equal(d.cpu().numpy(), od), (g.name, s)
            assert np.array_equal(p.cpu().numpy(), op), (g.name, s)
            if g is deep:
                assert (res[t]["launches"] == 1) == single, res[t]
        sv.close()
    Gd.free()
    Gs.free()
