"""Benchmark: direction-optimizing BFS on RMAT scale 24 (16 seeded sources).

One step = one BFS from each of the 16 sources through gbgpu_bfs (inputs and
outputs resident in HBM).  The JSON line reports Graph500 GTEPS (half the
degree sum of the reached vertices per second), the roofline of the round
kernel (algorithmic bytes / its HIP-event time, against 8 TB/s HBM), and the
oracle timed on the host as the CPU baseline.  Extra sections (weighted BFS,
the 3-D torus, batched queries, serving latency) are reported under "extra".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--scale 24]
       [--no-extra] [--no-cpu] [--only SECTION] [--serving-queries N]
       python bench.py --pmc-summary DIR | --trace-summary DIR
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, only if the kernel sources have not changed since."""
    import re
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if h and b and h.group(1) == kernel_source_hash():
        return float(b.group(1))
    return None


# the sources that decide what bfs_round_kernel reads and writes: the kernel,
# its shared device helpers, and the load-time structures it scans
ROUND_KERNEL_SOURCES = ("bfs.hip", "common.h", "emit.h", "graph.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ROUND_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1805_05208_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------------------
# Algorithmic byte model of one BFS (compulsory traffic of the method as run;
# random per-edge status probes are not counted)
# ---------------------------------------------------------------------------
def edge_keys(g):
    """Sorted (vertex << 32 | neighbour) keys of every stored edge, on the GPU
    (bookkeeping for the byte model only)."""
    import torch
    src = torch.repeat_interleave(torch.arange(g.n, device="cuda", dtype=torch.int64),
                                  torch.from_numpy(g.degrees()).cuda())
    return (src << 32) | torch.from_numpy(g.nbrs).cuda().to(torch.int64)


def parent_positions(g, keys, v, parent):
    import torch
    q = (torch.from_numpy(v.astype(np.int64)).cuda() << 32) | torch.from_numpy(
        parent[v].astype(np.int64)).cuda()
    return torch.searchsorted(keys, q).cpu().numpy() - g.offsets[v]


def bfs_bytes(g, keys, dist, parent, rlog):
    """Bytes of every round from the round log (direction, |U_r|, sum deg)
    and the outputs (which fix each dense scan's stopping point)."""
    n = g.n
    deg = g.degrees()
    INF = 2**31 - 1
    reach = dist != INF
    d = np.where(reach, dist, np.iinfo(np.int64).max).astype(np.int64)
    # position of the parent in v's ascending list (dense scans stop there)
    v = np.nonzero(reach & (parent != np.arange(n)))[0]
    pos = np.zeros(n, dtype=np.int64)
    pos[v] = parent_positions(g, keys, v, parent)
    # the rounds scan the vertices of degree >= 2; degree-1 vertices are
    # attached after the last round (8 B of list entries each, 4 B of their
    # neighbour's distance, 8 B of outputs when reached)
    nz = deg >= 2
    leaves = deg == 1
    leaf_bytes = 12 * int(leaves.sum()) + 8 * int((leaves & reach).sum())
    total = leaf_bytes
    per_round = []
    for r, (direction, cnt, edges, _q) in enumerate(rlog):
        cnt_next = rlog[r + 1][1] if r + 1 < len(rlog) else 0
        if direction == 2:  # dense
            # bitmaps V, F_r read and F_{r+1} written; each unvisited vertex
            # reads its 16-byte list head (first four neighbours); a scan
            # past the fourth neighbour also reads the offsets and 4 bytes
            # per further neighbour; dist and parent of the found vertices
            R = nz & (d > r)
            found = R & (d == r + 1)
            scan = np.where(found, pos + 1, deg)[R].astype(np.int64)
            beyond = scan > 4
            tail = int((16 + 4 * (scan[beyond] - 4)).sum())
            b = 3 * n // 8 + 16 * int(R.sum()) + tail + 8 * int(cnt_next)
        elif direction == 3:  # sparse from the bitmap
            b = n // 8 + 12 * int(cnt) + 4 * int(edges) + 16 * int(cnt_next)
        else:  # sparse from the queue
            b = 16 * int(cnt) + 4 * int(edges) + 16 * int(cnt_next)
        per_round.append(b)
        total += b
    return total, per_round


def host_cpu():
    """CPU model, logical CPU count and the CPUs this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def pinned_median(fn, reps=3):
    """Median wall time of fn() over reps runs with the calling thread pinned
    to one host CPU (the last one this process may use); the previous
    affinity is restored afterwards.  Returns (median seconds, cpu)."""
    allowed = sorted(os.sched_getaffinity(0))
    cpu = allowed[-1]
    os.sched_setaffinity(0, {cpu})
    try:
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
    finally:
        os.sched_setaffinity(0, set(allowed))
    return float(np.median(ts)), cpu


def oracle_all_cores(calls, threads):
    """Independent oracle queries, one per host thread (the oracle's C calls
    release the interpreter lock): (queries per second, wall seconds)."""
    import concurrent.futures as cf
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: c(), calls))
    wall = time.perf_counter() - t
    return len(calls) / wall, wall


def copy_peak_gbs(torch, nbytes=1 << 30, reps=5):
    """Streaming-copy rate of this GPU (read + write bytes of a 1 GiB device
    copy per second, best of reps, timed with HIP events)."""
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = 1e30
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--sources", type=int, default=16)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--opts", type=str, default="", help="JSON gbgpu_opts overrides")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--pmc-summary", type=str, default="",
                    help="print per-kernel averages of a rocprofv3 --pmc csv directory and exit")
    ap.add_argument("--trace-summary", type=str, default="",
                    help="print per-kernel totals and device concurrency of a rocprofv3 "
                         "--kernel-trace csv directory and exit")
    ap.add_argument("--segments", type=str, default="",
                    help="per-dispatch durations (kernel trace) or counter values (--pmc run) "
                         "of a rocprofv3 csv directory, in searches that start at --start; "
                         "print and exit")
    ap.add_argument("--start", type=str, default="bfs_init_kernel",
                    help="kernel that begins each search (with --segments)")
    ap.add_argument("--kernel", type=str, default="",
                    help="only dispatches of this kernel (with --segments)")
    ap.add_argument("--segment", type=int, default=-1,
                    help="print the dispatches of this search only (with --segments)")
    ap.add_argument("--counter", type=str, default="",
                    help="only this counter of a --pmc run (with --segments)")
    ap.add_argument("--step-log", type=str, default="",
                    help="a --only wbfs log: totals by kind of step (with --segments)")
    ap.add_argument("--serving-workers", type=int, default=8,
                    help="queries the server keeps on the device at once (worker streams)")
    ap.add_argument("--serving-queries", type=int, default=2000,
                    help="Poisson arrivals per offered load in the serving section")
    ap.add_argument("--torus", action="store_true",
                    help="with --only batched: the 256^3 torus instead of RMAT")
    ap.add_argument("--no-tuned", action="store_true",
                    help="ignore the autotuned options in paper_1805_05208_amd/tuned.json")
    ap.add_argument("--only", choices=["connectivity", "compressed", "wbfs", "sssp", "bc",
                                       "serving", "batched"],
                    default="",
                    help="time only the given section (for profiling) and print its own JSON line")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.segments:
        segments(args.segments, args.start, args.kernel, args.segment, args.step_log,
                 args.counter)
        return
    if args.torus and args.only != "batched":
        ap.error("--torus goes with --only batched")
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding a query over several GPUs is a design, not code that runs.", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen as gg
    import paper_1805_05208_amd as gb

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    gb.lib()
    user_opts = json.loads(args.opts) if args.opts else {}
    tuned_path = TUNED

    t = time.time()
    gname = "torus256" if args.torus else f"rmat{args.scale}"
    g = gg.torus3d(256) if args.torus else gg.rmat(args.scale, seed=1)
    srcs = [int(s) for s in gg.sources(g, args.sources, seed=3)]
    log(f"generated {gname}: n={g.n} m={g.m} in {time.time() - t:.1f}s")
    G = gb.Graph.from_csr(g, validate=False, with_weights=False)
    deg = g.degrees()
    stream = torch.cuda.current_stream()
    if args.only in ("wbfs", "sssp", "bc"):
        # one section on the same graph and the first four sources: weighted
        # BFS, Bellman-Ford and widest path (weights in [1, 24)), or
        # betweenness; --warmup untimed then --steps timed passes
        srcs4 = srcs[:4]
        if args.only == "bc":
            runs = [("betweenness", lambda s: gb.betweenness(G, s), G)]
        else:
            Gw = gb.Graph(G.offsets, G.nbrs, gg.weights(g, 24, seed=2), validate=False)
            if args.only == "wbfs":
                runs = [("wbfs", lambda s: gb.wbfs(Gw, s), Gw)]
            else:
                runs = [("bellman_ford", lambda s: gb.bellman_ford(Gw, s), Gw),
                        ("widest_path", lambda s: gb.widest_path(Gw, s), Gw)]
        res = {"metric": f"{args.only}_section", "config": {"workload": f"rmat{args.scale}",
                                                             "sources": len(srcs4)}}
        edges = 0
        for s in srcs4:
            d, _ = gb.bfs(G, s)
            edges += int(deg[d.cpu().numpy() != 2**31 - 1].sum()) // 2
        if args.only == "wbfs":
            # the step log of one search per source (bucket, entries, degree
            # sum, kind: 0 push, 1 mark, 2 pull), in launch order, for
            # joining with a kernel trace
            logs = {}
            for s in srcs4:
                gb.wbfs(Gw, s)
                logs[str(s)] = Gw.wbfs_log().tolist()
            res["step_logs"] = logs
        for key, fn, _gr in runs:
            for _ in range(args.warmup):
                for s in srcs4:
                    fn(s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                for s in srcs4:
                    fn(s)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / max(args.steps, 1)
            res[f"{key}_ms_per_source"] = round(dt * 1e3 / len(srcs4), 3)
            res[f"{key}_gteps"] = round(edges / dt / 1e9, 2)
            log(f"{key}: {res[f'{key}_ms_per_source']} ms/source, {res[f'{key}_gteps']} GTEPS")
        print(json.dumps(res), flush=True)
        return
    if args.only == "compressed":
        # compressed adjacency: size, then BFS over the compressed lists and
        # the same rounds over the plain lists, --steps timed passes over
        # the sources
        nbytes = gb.compress(G)
        res = {"metric": "compressed_section", "config": {"workload": f"rmat{args.scale}",
                                                           "sources": len(srcs)},
               "compressed_bytes": nbytes,
               "list_bytes_per_edge": round((nbytes - 8 * (g.n + 1)) / g.m, 3)}
        edges = 0
        for s in srcs:
            d, _ = gb.bfs(G, s)
            edges += int(deg[d.cpu().numpy() != 2**31 - 1].sum()) // 2
        for key, fn in (("bfs_compressed", gb.bfs_compressed), ("bfs_simple", gb.bfs_simple)):
            for _ in range(args.warmup):
                for s in srcs:
                    fn(G, s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                for s in srcs:
                    fn(G, s)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / max(args.steps, 1)
            res[f"{key}_gteps"] = round(edges / dt / 1e9, 2)
            res[f"{key}_ms_per_source"] = round(dt * 1e3 / len(srcs), 3)
            log(f"{key}: {res[f'{key}_ms_per_source']} ms/source, {res[f'{key}_gteps']} GTEPS")
        print(json.dumps(res), flush=True)
        return
    if args.only == "batched":
        # 64 seeded sources in one gbgpu_bfs_multi call against the same
        # sources one gbgpu_bfs call each; --steps timed repetitions
        s64 = [int(x) for x in gg.sources(g, 64, seed=3)]
        gb.bfs(G, s64[0])
        D, P = gb.bfs_multi(G, s64)
        d1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
        p1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
        res = {"metric": "batched_section", "config": {"workload": gname, "sources": 64}}
        for key, fn in (("batched64", lambda: gb.bfs_multi(G, s64, dist=D, parent=P)),
                        ("single", lambda: [gb.bfs(G, s, dist=d1, parent=p1) for s in s64])):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / max(args.steps, 1)
            res[f"{key}_ms"] = round(dt * 1e3, 3)
            res[f"{key}_qps"] = round(64 / dt, 1)
            log(f"{key}: {dt * 1e3:.3f} ms for 64 sources, {64 / dt:.1f} q/s")
        print(json.dumps(res), flush=True)
        return
    if args.only == "serving":
        res = {"metric": "serving_section", "config": {"workload": "six resident graphs"}}
        res.update(run_serving(g, G, gg, gb, torch, nq=args.serving_queries,
                               cpu=not args.no_cpu, workers=args.serving_workers))
        print(json.dumps(res), flush=True)
        return
    if args.only == "connectivity":
        # LDD (beta 0.2) and connectivity on the same graph: warmup, then
        # --steps timed calls of each
        res = {"metric": "connectivity_section", "config": {"workload": f"rmat{args.scale}",
                                                             "beta": 0.2}}
        for key, fn in (("ldd", gb.ldd), ("connectivity", gb.connectivity)):
            _, st = fn(G, 0.2, 1, stats=True)
            for _ in range(args.warmup):
                fn(G, 0.2, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn(G, 0.2, 1)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
            res[f"{key}_ms"] = round(ms, 3)
            res[f"{key}_rounds"] = st["rounds"]
            res[f"{key}_clusters"] = st["reached"]
            log(f"{key}: {ms:.3f} ms, {st['rounds']} rounds/levels, {st['reached']} clusters/components")
        print(json.dumps(res), flush=True)
        return
    if not args.opts and not args.no_tuned:
        from paper_1805_05208_amd import autotune
        _, _, st0 = gb.bfs(G, srcs[0], stats=True)
        sig = autotune.signature(g.n, g.m, int(deg.max()), st0["rounds"])
        tuned = autotune.lookup(tuned_path, sig, "bfs")
        if tuned:
            user_opts = dict(tuned)
            log(f"using autotuned options for {sig}: {tuned}")

    # --- correctness spot check + per-source edge counts -------------------
    half_edges = []
    outs = []
    for s in srcs:
        d, p = gb.bfs(G, s)
        dn = d.cpu().numpy()
        half_edges.append(int(deg[dn != 2**31 - 1].sum()) // 2)
        outs.append((dn, p.cpu().numpy(), G.bfs_log()))
    step_edges = sum(half_edges)

    if args.copy_probe:
        copy_probe(torch)
    # --- warmup + timed steps ------------------------------------------------
    # output buffers are allocated once, like the graph
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    # a step is the 16 searches one after another in one library call
    # (gbgpu_bfs_many: the next search starts when the device reports the
    # previous one done, without a return to Python in between)
    for _ in range(args.warmup):
        gb.bfs_many(G, srcs, dist=dist, parent=parent, row_stride=0, opts=user_opts)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        gb.bfs_many(G, srcs, dist=dist, parent=parent, row_stride=0, opts=user_opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / args.steps
    gteps = step_edges * args.steps / wall / 1e9
    log(f"BFS: {ms_per_step:.3f} ms/step ({len(srcs)} sources), {gteps:.1f} GTEPS, "
        f"event time {gpu_ms / args.steps:.3f} ms/step")
    # the same steps with one gbgpu_bfs call per source from Python, for
    # comparison (not the headline)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for s in srcs:
            gb.bfs(G, s, dist=dist, parent=parent, opts=user_opts)
    torch.cuda.synchronize()
    per_call_gteps = step_edges * args.steps / (time.perf_counter() - t1) / 1e9
    log(f"BFS with one call per source: {per_call_gteps:.1f} GTEPS")
    # each source timed on its own: median of 5 calls, HIP events on the
    # stream around each call (per-source GTEPS and their harmonic mean)
    per_src_ms = []
    for s in srcs:
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gb.bfs(G, s, dist=dist, parent=parent, opts=user_opts)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        per_src_ms.append(float(np.median(ts)))
    per_src_gteps = [he / (ms * 1e-3) / 1e9 for he, ms in zip(half_edges, per_src_ms)]
    hmean_gteps = len(per_src_gteps) / sum(1.0 / x for x in per_src_gteps)
    log(f"per-source GTEPS (median of 5 each): min {min(per_src_gteps):.1f} max "
        f"{max(per_src_gteps):.1f}, harmonic mean {hmean_gteps:.1f}")
    copy_gbs = copy_peak_gbs(torch)
    log(f"streaming copy: {copy_gbs:.0f} GB/s (read + write)")

    # --- the same steps again, each BFS's round-kernel launches bracketed by
    # two HIP events on the library's stream (profile=1).  Reading the events
    # needs a host sync per BFS, which the timed pass above avoids; the work
    # is identical.
    popts = dict(user_opts)
    popts["profile"] = 1
    kernel_ms = 0.0
    launches = 0
    for _ in range(args.steps):
        for s in srcs:
            _, _, st = gb.bfs(G, s, dist=dist, parent=parent, opts=popts, stats=True)
            kernel_ms += st["kernel_ms"]
            launches += st["launches"]
    log(f"round kernels: {kernel_ms / args.steps:.3f} ms/step over {launches // args.steps} "
        f"launches")

    # --- roofline of the round kernel ---------------------------------------
    keys = edge_keys(g)
    bytes_per_bfs = []
    for (dn, pn, rl) in outs:
        b, _ = bfs_bytes(g, keys, dn, pn, rl)
        bytes_per_bfs.append(b)
    del keys
    alg_bytes = sum(bytes_per_bfs) * args.steps
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else None
    roof = {
        "kernel": "gb::bfs_round_kernel",
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": None,
        "bytes_per_launch": alg_bytes / max(launches, 1),
        "avg_launch_us": kernel_ms * 1e3 / max(launches, 1),
        "launches": launches,
        # the same bytes against the measured streaming-copy rate, and over
        # the whole step's wall time (init, tails and gaps included)
        "copy_peak_gbs": round(copy_gbs, 1),
        "frac_of_copy_peak": round(achieved / copy_gbs, 4) if achieved else None,
        "frac_wall": round(alg_bytes / (wall * 1e9) / HBM_PEAK_GBS, 4),
    }
    roof["traffic"] = measured_traffic("bfs_round_kernel_rmat24_traffic.md")

    # --- CPU baseline: the oracle on a bounded sample ---------------------------
    # sequential C oracle (-O3), one thread pinned to one host CPU, median of
    # 3 runs per source, two of the timed sources (about 25 s on the host)
    cpu = None
    if not args.no_cpu:
        import oracle
        nsamp = 2
        meds = []
        pin = None
        for i in range(nsamp):
            od, op = oracle.bfs(g, srcs[i])
            assert np.array_equal(od, outs[i][0]) and np.array_equal(op, outs[i][1]), \
                "GPU BFS differs from the oracle"
            t_med, pin = pinned_median(lambda: oracle.bfs(g, srcs[i]), reps=3)
            meds.append(t_med)
        ct = sum(meds)
        hc = host_cpu()
        cpu = {"value": round(sum(half_edges[:nsamp]) / ct / 1e9, 4), "unit": "GTEPS", "cores": 1,
               "kind": "oracle",
               "sample": f"sequential BFS + min-ID parent pass (C, -O3) from {nsamp} of the "
                         f"{len(srcs)} sources on rmat{args.scale}, median of 3 runs each, "
                         f"thread pinned to CPU {pin} ({ct:.1f} s of medians)",
               "host_cpu": hc["model"], "host_nproc": hc["nproc"],
               "host_cpus_allowed": hc["affinity"]}
        log(f"oracle: {cpu['value']} GTEPS on one pinned core of {hc['model']} "
            f"({hc['nproc']} CPUs); GPU results identical on the sample")

    extra = {}
    if not args.no_extra:
        extra = run_extras(g, G, srcs, gg, gb, torch, user_opts)

    line = {
        "metric": "GTEPS (direction-optimizing BFS, 1 GPU)",
        "value": round(gteps, 2),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"BFS rmat{args.scale} ef16 (0.57,0.19,0.19,0.05) symmetrized, "
                               f"{len(srcs)} seeded sources per step (one gbgpu_bfs_many call)",
                   "n": g.n, "m_directed": g.m, "sources": len(srcs),
                   "edges_per_step_graph500": step_edges, "parallelism": "1 GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "opts": user_opts,
        "gteps_one_call_per_source": round(per_call_gteps, 2),
        "per_source_gteps": [round(x, 1) for x in per_src_gteps],
        "per_source_ms": [round(x, 4) for x in per_src_ms],
        "harmonic_mean_gteps": round(hmean_gteps, 2),
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


COPY_PROBE_BYTES = 1 << 30


def copy_probe(torch):
    """A plain device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB), run
    three times, whose FETCH_SIZE / WRITE_SIZE readings convert the counters
    into bytes."""
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y


def pmc_summary(path):
    """Mean counter value per dispatch, by kernel, from the counter_collection
    csv files rocprofv3 wrote under `path` (FETCH_SIZE and WRITE_SIZE are in
    KiB)."""
    import csv
    import glob
    from collections import defaultdict
    acc = defaultdict(lambda: [0.0, set()])
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = (row["Kernel_Name"].split("(")[0][:90], row["Counter_Name"])
                acc[k][0] += float(row["Counter_Value"])
                acc[k][1].add(row["Dispatch_Id"])
    for (kern, ctr), (tot, ids) in sorted(acc.items(), key=lambda kv: -kv[1][0]):
        print(f"{ctr:12s} dispatches={len(ids):6d} mean={tot / len(ids):14.1f}  {kern}")


def trace_summary(path, window_s=1.0):
    """Kernel time by kernel, and how much kernels overlapped on the device,
    from the kernel_trace csv files rocprofv3 wrote under `path`:
    concurrency = sum of kernel durations / time at least one kernel ran,
    overall and per window of `window_s` seconds."""
    import csv
    import glob
    from collections import defaultdict
    per = defaultdict(lambda: [0, 0])
    iv = []
    for f in glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
                k = row["Kernel_Name"].split("(")[0][:70]
                per[k][0] += 1
                per[k][1] += b - a
                iv.append((a, b))
    if not iv:
        print("no kernel trace under", path)
        return
    iv.sort()
    t0, t1 = iv[0][0], max(b for _, b in iv)
    tot = sum(b - a for a, b in iv)
    print(f"{len(iv)} kernels over {(t1 - t0) / 1e9:.3f} s, {tot / 1e9:.3f} s of kernel time")
    for k, (n, ns) in sorted(per.items(), key=lambda kv: -kv[1][1])[:16]:
        print(f"  {k:70s} calls={n:8d} total={ns / 1e6:10.2f} ms avg={ns / n / 1e3:9.2f} us "
              f"{100.0 * ns / tot:5.1f} %")
    # busy time (union of the intervals), overall and per window
    w = int(window_s * 1e9)
    nwin = (t1 - t0) // w + 1
    busy = [0] * nwin
    work = [0] * nwin
    for a, b in iv:
        x = a
        while x < b:
            i = (x - t0) // w
            e = min(b, t0 + (i + 1) * w)
            work[i] += e - x
            x = e
    cur_a, cur_b = iv[0]
    merged = []
    for a, b in iv[1:]:
        if a > cur_b:
            merged.append((cur_a, cur_b))
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    merged.append((cur_a, cur_b))
    for a, b in merged:
        x = a
        while x < b:
            i = (x - t0) // w
            e = min(b, t0 + (i + 1) * w)
            busy[i] += e - x
            x = e
    tb = sum(busy)
    print(f"device busy {tb / 1e9:.3f} s ({100.0 * tb / (t1 - t0):.1f} % of the span), "
          f"mean concurrency {tot / max(tb, 1):.2f}")
    print("window  busy%  concurrency")
    for i in range(nwin):
        if busy[i]:
            print(f"{i * window_s:6.0f}  {100.0 * busy[i] / w:5.1f}  {work[i] / busy[i]:6.2f}")


def segments(path, start, kernel="", which=-1, step_log="", counter=""):
    """Dispatches of a rocprofv3 run in Dispatch_Id order, cut into searches
    at each dispatch of `start`: per dispatch its duration in us (a
    kernel_trace csv) or its counter value summed over the counters and
    dimensions collected, or of `counter` alone (a counter_collection csv),
    kernel names without arguments.  With a step log (the JSON line of `bench.py --only wbfs`,
    whose step_logs come in search order from the first search), the
    weighted-BFS step dispatches of each logged search are totalled by kind
    of step (push / mark / pull)."""
    import csv
    import glob
    from collections import OrderedDict
    rows = []
    for pat in ("*kernel_trace.csv", "*counter_collection.csv"):
        for f in glob.glob(os.path.join(path, "**", pat), recursive=True):
            with open(f) as fh:
                rows += [(pat, r) for r in csv.DictReader(fh)]
    disp = OrderedDict()
    for pat, r in sorted(rows, key=lambda pr: int(pr[1]["Dispatch_Id"])):
        d = int(r["Dispatch_Id"])
        name = r["Kernel_Name"].split("(")[0]
        if pat.startswith("*kernel"):
            disp[d] = [name, (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3]
        elif not counter or r["Counter_Name"] == counter:
            disp.setdefault(d, [name, 0.0])[1] += float(r["Counter_Value"])
    segs = []
    for name, v in disp.values():
        if start in name:
            segs.append([])
        if segs and (not kernel or kernel in name):
            segs[-1].append((name, v))
    unit = "us" if rows and rows[0][0].startswith("*kernel") else "counter"
    print(f"{len(segs)} searches starting at {start}; values in {unit}")
    for i, sg in enumerate(segs):
        if which >= 0 and i != which:
            continue
        tot = sum(v for _, v in sg)
        print(f"search {i}: {len(sg)} dispatches, total {tot:.1f}")
        if which >= 0:
            for j, (name, v) in enumerate(sg):
                print(f"  {j:5d} {name:40s} {v:14.1f}")
    if step_log:
        with open(step_log) as fh:
            line = [x for x in fh if x.startswith('{"metric"')][-1]
        logs = json.loads(line)["step_logs"]
        for i, (src, lg) in enumerate(logs.items()):
            steps = [v for name, v in segs[i] if "wbfs_step_kernel" in name][:len(lg)]
            tot = {}
            for (_b, _c, _e, mode), v in zip(lg, steps):
                k = ("push", "mark", "pull")[mode]
                n, x = tot.get(k, (0, 0.0))
                tot[k] = (n + 1, x + v)
            print(f"source {src}: {len(lg)} steps; " + ", ".join(
                f"{k} {n} steps {x:.1f}" for k, (n, x) in tot.items()))


TUNED = os.path.join(ROOT, "paper_1805_05208_amd", "tuned.json")


def tuned_opts(gb, G, g, src, kind):
    """Autotuned options stored for this graph's signature, if any."""
    from paper_1805_05208_amd import autotune
    run = gb.bfs if kind == "bfs" else gb.wbfs
    _, _, st = run(G, src, stats=True)
    sig = autotune.signature(g.n, g.m, int(g.degrees().max()), st["rounds"])
    return autotune.lookup(TUNED, sig, kind)


def timed(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def run_extras(g, G, srcs, gg, gb, torch, user_opts):
    extra = {}
    deg = g.degrees()
    # RMAT scale 16: one BFS from the first seeded source, median of 100
    # calls after 5 warm-ups (HIP events around each call); the whole graph
    # fits in L2 and the Infinity Cache, so its roofline fraction (byte
    # model over the call's time) is context, not a target
    try:
        g16 = gg.rmat(16, seed=1)
        G16 = gb.Graph.from_csr(g16, validate=False, with_weights=False)
        s16 = int(gg.sources(g16, 1, seed=3)[0])
        d16 = torch.empty(g16.n, dtype=torch.int32, device="cuda")
        p16 = torch.empty(g16.n, dtype=torch.int32, device="cuda")
        o16 = tuned_opts(gb, G16, g16, s16, "bfs") or {}
        extra["rmat16_opts"] = o16
        _, _, st16 = gb.bfs(G16, s16, dist=d16, parent=p16, opts=o16, stats=True)
        dn, pn = d16.cpu().numpy(), p16.cpu().numpy()
        he16 = int(g16.degrees()[dn != 2**31 - 1].sum()) // 2
        b16, _ = bfs_bytes(g16, edge_keys(g16), dn, pn, G16.bfs_log())
        stream = torch.cuda.current_stream()
        for _ in range(5):
            gb.bfs(G16, s16, dist=d16, parent=p16, opts=o16)
        ts = []
        for _ in range(100):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gb.bfs(G16, s16, dist=d16, parent=p16, opts=o16)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms16 = float(np.median(ts))
        extra["rmat16_bfs_ms"] = round(ms16, 4)
        extra["rmat16_bfs_gteps"] = round(he16 / (ms16 * 1e-3) / 1e9, 2)
        extra["rmat16_bfs_rounds"] = st16["rounds"]
        extra["rmat16_bfs_frac_model"] = round(b16 / (ms16 * 1e-3) / 8e12, 4)
        log(f"BFS rmat16: {ms16 * 1e3:.1f} us (median of 100), {extra['rmat16_bfs_gteps']} GTEPS, "
            f"{st16['rounds']} rounds, model fraction {extra['rmat16_bfs_frac_model']}")
        del G16
    except Exception as ex:  # noqa: BLE001 - extras must not hide the headline
        extra["error_rmat16"] = repr(ex)[:300]
    # two searches in flight (beside the sequential headline, never instead
    # of it): a second handle on the same CSR arrays has its own workspace;
    # two host threads each run half of the 16 sources back to back on a
    # stream of their own, so one search's small rounds and tail launches
    # overlap the other's dense rounds
    try:
        import threading
        G2 = gb.Graph(G.offsets, G.nbrs, None, validate=False)
        he = []
        for s in srcs:
            d, _ = gb.bfs(G, s, opts=user_opts)
            he.append(int(deg[d.cpu().numpy() != 2**31 - 1].sum()) // 2)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        bufs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"),
                 torch.empty(g.n, dtype=torch.int32, device="cuda")) for _ in range(2)]
        lat = [[], []]

        def half(i, record):
            H = (G, G2)[i]
            d, p = bufs[i]
            for s in srcs[i::2]:
                t = time.perf_counter()
                gb.bfs(H, s, dist=d, parent=p, opts=user_opts, stream=streams[i])
                if record:
                    lat[i].append(time.perf_counter() - t)

        def both(record):
            th = [threading.Thread(target=half, args=(i, record)) for i in range(2)]
            for x in th:
                x.start()
            for x in th:
                x.join()
            torch.cuda.synchronize()

        both(False)
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            both(True)
        wall = time.perf_counter() - t0
        # each thread's last search against the same search on its own
        same = True
        for i in range(2):
            d0, p0 = gb.bfs(G, srcs[i::2][-1], opts=user_opts)
            same &= bool(torch.equal(d0, bufs[i][0])) and bool(torch.equal(p0, bufs[i][1]))
        extra["bfs_two_in_flight_gteps"] = round(sum(he) * reps / wall / 1e9, 1) if same else None
        extra["bfs_two_in_flight_ms_per_search"] = round(1e3 * float(np.median(lat[0] + lat[1])), 3)
        log(f"BFS, two searches in flight: {extra['bfs_two_in_flight_gteps']} GTEPS, "
            f"{extra['bfs_two_in_flight_ms_per_search']} ms per search (median)")
        G2.free()
    except Exception as ex:  # noqa: BLE001 - extras must not hide the headline
        extra["error_two_in_flight"] = repr(ex)[:300]
    # weighted BFS on the same graph, w in [1, 24)
    try:
        w = gg.weights(g, 24, seed=2)
        Gw = gb.Graph(G.offsets, G.nbrs, w, validate=False)
        # the weighted search takes its own tuned options (none: the
        # library's defaults), not the BFS ones
        wopts = tuned_opts(gb, Gw, g, srcs[0], "wbfs")
        extra["wbfs_rmat24_opts"] = wopts
        # every one of the 16 sources: GTEPS, buckets, and the fraction of
        # the HBM roofline by the byte model of a weighted search (8 bytes
        # per list entry of the reached component, neighbour and weight,
        # plus 24 per vertex for init and finalize)
        tot_e, tot_t, nb = 0, 0.0, 0
        for s in srcs:
            d, p, st = gb.wbfs(Gw, s, opts=wopts, stats=True)
            e = int(deg[gb.as_u32(d) != 0xFFFFFFFF].sum()) // 2
            t = timed(lambda: gb.wbfs(Gw, s, opts=wopts), reps=2)
            tot_e += e
            tot_t += t
            nb += st["rounds"]
        ns = len(srcs)
        extra["wbfs_rmat24_sources"] = ns
        extra["wbfs_rmat24_gteps"] = round(tot_e / tot_t / 1e9, 2)
        extra["wbfs_rmat24_ms"] = round(tot_t * 1e3 / ns, 3)
        extra["wbfs_rmat24_buckets"] = round(nb / ns, 1)
        extra["wbfs_rmat24_frac_model"] = round((16 * tot_e + 24 * g.n * ns) / tot_t / 8e12, 4)
        log(f"wBFS rmat: {extra['wbfs_rmat24_gteps']} GTEPS, {extra['wbfs_rmat24_ms']} ms/source "
            f"over {ns} sources, {nb / ns:.1f} buckets, model fraction "
            f"{extra['wbfs_rmat24_frac_model']}")
        # general-weight SSSP (Bellman-Ford rounds) and widest path on the
        # same weighted graph and sources (edges of the reached component,
        # as for wBFS)
        for key, fn, reached in (
                ("bellman_ford", gb.bellman_ford, lambda x: x.cpu().numpy() != 2**63 - 1),
                ("widest_path", gb.widest_path, lambda x: gb.as_u32(x) != 0)):
            tot_e, tot_t, rounds = 0, 0.0, 0
            for s in srcs[:4]:
                x, st = fn(Gw, s, stats=True)
                rounds += st["rounds"]
                tot_e += int(deg[reached(x)].sum()) // 2
                tot_t += timed(lambda: fn(Gw, s), reps=2)
            extra[f"{key}_rmat24_gteps"] = round(tot_e / tot_t / 1e9, 2)
            extra[f"{key}_rmat24_ms"] = round(tot_t * 1e3 / 4, 3)
            extra[f"{key}_rmat24_rounds"] = round(rounds / 4, 1)
            log(f"{key} rmat: {extra[f'{key}_rmat24_gteps']} GTEPS, "
                f"{extra[f'{key}_rmat24_ms']} ms/source, {rounds / 4:.1f} rounds")
        # single-source betweenness (forward + backward pass over the BFS
        # levels; every edge of the reached component is visited twice)
        tot_e, tot_t = 0, 0.0
        for s in srcs[:4]:
            x, st = gb.betweenness(G, s, stats=True)
            d, _ = gb.bfs(G, s)
            tot_e += int(deg[d.cpu().numpy() != 2**31 - 1].sum()) // 2
            tot_t += timed(lambda: gb.betweenness(G, s), reps=2)
        extra["bc_rmat24_ms"] = round(tot_t * 1e3 / 4, 3)
        extra["bc_rmat24_gteps"] = round(tot_e / tot_t / 1e9, 2)
        log(f"betweenness rmat: {extra['bc_rmat24_ms']} ms/source, {extra['bc_rmat24_gteps']} GTEPS")
        # compressed adjacency: size, and the same simple rounds over the
        # compressed and over the plain lists (same sources as the headline)
        nbytes = gb.compress(G)
        extra["compressed_rmat24_list_bytes_per_edge"] = round((nbytes - 8 * (g.n + 1)) / g.m, 3)
        extra["compressed_rmat24_bytes"] = nbytes
        e4 = 0
        for s in srcs[:4]:
            d, _ = gb.bfs(G, s)
            e4 += int(deg[d.cpu().numpy() != 2**31 - 1].sum()) // 2
        for key, fn in (("bfs_compressed", gb.bfs_compressed), ("bfs_simple", gb.bfs_simple)):
            tot_t = 0.0
            for s in srcs[:4]:
                tot_t += timed(lambda: fn(G, s), reps=2)
            extra[f"{key}_rmat24_gteps"] = round(e4 / tot_t / 1e9, 2)
            extra[f"{key}_rmat24_ms"] = round(tot_t * 1e3 / 4, 3)
            log(f"{key} rmat: {extra[f'{key}_rmat24_ms']} ms/source, {extra[f'{key}_rmat24_gteps']} GTEPS")
        log(f"compressed lists: {extra['compressed_rmat24_list_bytes_per_edge']} B/edge "
            f"(plain 4), {nbytes / 1e9:.2f} GB with offsets")
        # low-diameter decomposition and connectivity (beta 0.2): whole graph
        for key, fn in (("ldd", gb.ldd), ("connectivity", gb.connectivity)):
            _, st = fn(G, 0.2, 1, stats=True)
            t = timed(lambda: fn(G, 0.2, 1), reps=3)
            extra[f"{key}_rmat24_ms"] = round(t * 1e3, 3)
            extra[f"{key}_rmat24_gteps"] = round(g.m / 2 / t / 1e9, 2)
            extra[f"{key}_rmat24_rounds"] = st["rounds"]
            log(f"{key} rmat: {extra[f'{key}_rmat24_ms']} ms, {extra[f'{key}_rmat24_gteps']} GTEPS, "
                f"{st['rounds']} rounds/levels, {st['reached']} clusters/components")
        # batched: 64 sources in one call vs one at a time
        s64 = [int(x) for x in gg.sources(g, 64, seed=3)]
        tb = timed(lambda: gb.bfs_multi(G, s64), reps=2)
        D0, P0 = gb.bfs_multi(G, s64)
        D1, P1 = gb.bfs_multi(G, s64, opts={"persistent": 1})
        same = bool(torch.equal(D0, D1)) and bool(torch.equal(P0, P1))
        del D1, P1
        tp = timed(lambda: gb.bfs_multi(G, s64, dist=D0, parent=P0, opts={"persistent": 1}),
                   reps=2)
        del D0, P0
        t1 = timed(lambda: [gb.bfs(G, s) for s in s64[:16]], reps=1) * 4
        extra["batched64_qps"] = round(64 / tb, 1)
        extra["batched64_persistent_qps"] = round(64 / tp, 1) if same else None
        extra["single_qps"] = round(64 / t1, 1)
        log(f"batched 64: {extra['batched64_qps']} q/s ({extra['batched64_persistent_qps']} as one "
            f"persistent launch) vs one-at-a-time {extra['single_qps']} q/s")
        # the oracle on every host core: independent BFS queries of the
        # batch, one per thread
        import oracle
        thr = min(16, len(os.sched_getaffinity(0)))
        qps, wall = oracle_all_cores([lambda s=s: oracle.bfs(g, s) for s in s64[:thr]], thr)
        extra["oracle_all_cores_batched_qps"] = round(qps, 3)
        extra["oracle_all_cores_threads"] = thr
        log(f"oracle on {thr} host threads: {qps:.2f} BFS/s on rmat24 ({wall:.1f} s)")
        del Gw
    except Exception as ex:  # noqa: BLE001 - extras must not hide the headline
        extra["error_rmat"] = repr(ex)[:300]
    try:
        tg = gg.torus3d(256).with_weights(24, seed=2)
        T = gb.Graph.from_csr(tg, validate=False)
        ts = int(gg.sources(tg, 1, seed=3)[0])
        topt_b = tuned_opts(gb, T, tg, ts, "bfs") or user_opts
        topt_w = tuned_opts(gb, T, tg, ts, "wbfs")
        tt = timed(lambda: gb.bfs(T, ts, opts=topt_b), reps=2)
        # weighted BFS from 16 seeded sources (every vertex is reached)
        t16 = [int(x) for x in gg.sources(tg, 16, seed=3)]
        tw, nb = 0.0, 0
        for s in t16:
            _, _, st = gb.wbfs(T, s, opts=topt_w, stats=True)
            nb += st["rounds"]
            tw += timed(lambda: gb.wbfs(T, s, opts=topt_w), reps=1)
        tw /= len(t16)
        extra["torus256_opts"] = {"bfs": topt_b, "wbfs": topt_w}
        extra["torus256_bfs_ms"] = round(tt * 1e3, 3)
        extra["torus256_bfs_gteps"] = round(tg.m / 2 / tt / 1e9, 3)
        extra["torus256_wbfs_sources"] = len(t16)
        extra["torus256_wbfs_ms"] = round(tw * 1e3, 3)
        extra["torus256_wbfs_gteps"] = round(tg.m / 2 / tw / 1e9, 3)
        extra["torus256_wbfs_buckets"] = round(nb / len(t16), 1)
        extra["torus256_wbfs_frac_model"] = round((8 * tg.m + 24 * tg.n) / tw / 8e12, 4)
        log(f"torus: BFS {extra['torus256_bfs_ms']} ms, wBFS {extra['torus256_wbfs_ms']} ms per "
            f"source over {len(t16)} sources ({nb / len(t16):.0f} buckets)")
        # (library defaults: the BFS-tuned options would set the direction
        # threshold the relaxation rounds choose for themselves)
        tbf = timed(lambda: gb.bellman_ford(T, ts), reps=1)
        twp = timed(lambda: gb.widest_path(T, ts), reps=1)
        tbc = timed(lambda: gb.betweenness(T, ts), reps=1)
        for key, fn in (("ldd", gb.ldd), ("connectivity", gb.connectivity)):
            t = timed(lambda: fn(T, 0.2, 1), reps=2)
            extra[f"torus256_{key}_ms"] = round(t * 1e3, 3)
            log(f"torus: {key} {extra[f'torus256_{key}_ms']} ms")
        extra["torus256_bc_ms"] = round(tbc * 1e3, 3)
        extra["torus256_bellman_ford_ms"] = round(tbf * 1e3, 3)
        extra["torus256_widest_path_ms"] = round(twp * 1e3, 3)
        log(f"torus: Bellman-Ford {extra['torus256_bellman_ford_ms']} ms, "
            f"widest path {extra['torus256_widest_path_ms']} ms, "
            f"betweenness {extra['torus256_bc_ms']} ms")
        # batched on the high-diameter graph: 64 sources in one call against
        # the same 64 one at a time (4 timed, scaled)
        t64 = [int(x) for x in gg.sources(tg, 64, seed=3)]
        tb = timed(lambda: gb.bfs_multi(T, t64), reps=1)
        t1 = timed(lambda: [gb.bfs(T, s) for s in t64[:4]], reps=1) * 16
        extra["torus256_batched64_qps"] = round(64 / tb, 1)
        extra["torus256_single_qps"] = round(64 / t1, 1)
        log(f"torus batched 64: {extra['torus256_batched64_qps']} q/s vs one-at-a-time "
            f"{extra['torus256_single_qps']} q/s")
        del T
    except Exception as ex:  # noqa: BLE001
        extra["error_torus"] = repr(ex)[:300]
    try:
        extra.update(run_uneven_batch(gg, gb))
    except Exception as ex:  # noqa: BLE001
        extra["error_uneven"] = repr(ex)[:300]
    try:
        extra.update(run_serving(g, G, gg, gb, torch))
    except Exception as ex:  # noqa: BLE001
        extra["error_serving"] = repr(ex)[:300]
    return extra


def run_uneven_batch(gg, gb):
    """256 BFS queries over 8 RMAT graphs of scales 12..20 (edge factor 16),
    32 per graph, in one gbgpu_bfs_batch call, against the same queries one
    at a time through gbgpu_bfs."""
    scales = [12, 13, 14, 15, 16, 17, 18, 20]
    graphs = [gg.rmat(sc, seed=1) for sc in scales]
    Gs = [gb.Graph.from_csr(gr, validate=False, with_weights=False) for gr in graphs]
    qg, qs = [], []
    for i, gr in enumerate(graphs):
        for s in gg.sources(gr, 32, seed=3):
            qg.append(Gs[i])
            qs.append(int(s))
    tb = timed(lambda: gb.bfs_batch(qg, qs), reps=2)
    # the same batch as one persistent launch (every round of every group
    # behind grid barriers), checked equal to the default form
    D0, P0 = gb.bfs_batch(qg, qs)
    D1, P1 = gb.bfs_batch(qg, qs, opts={"persistent": 1})
    same = all(bool((a == b).all()) for a, b in zip(D0 + P0, D1 + P1))
    tp = timed(lambda: gb.bfs_batch(qg, qs, opts={"persistent": 1}), reps=2)
    t1 = timed(lambda: [gb.bfs(Gq, s) for Gq, s in zip(qg, qs)], reps=2)
    out = {"uneven256_batched_qps": round(len(qs) / tb, 1),
           "uneven256_persistent_qps": round(len(qs) / tp, 1) if same else None,
           "uneven256_single_qps": round(len(qs) / t1, 1)}
    log(f"uneven batch of 256 over RMAT 12..20: {out['uneven256_batched_qps']} q/s batched "
        f"({out['uneven256_persistent_qps']} as one persistent launch) vs "
        f"{out['uneven256_single_qps']} q/s one at a time")
    for G_ in Gs:
        G_.free()
    return out


class ServedMix:
    """Drives the server with a seeded mix of BFS / weighted BFS queries on
    the resident graphs.  Each in-flight query has its own output pair from
    a per-graph pool; a pair is reused only after its ticket was polled, its
    status checked and its outputs verified against the standalone call
    (a digest of dist and parent for every query; element by element for
    the queries whose source is one of the first two of its graph)."""

    POOL = 24
    NSRC = 32

    def __init__(self, graphs, sv, ids, gg, gb, torch):
        self.graphs, self.sv, self.ids, self.gb, self.torch = graphs, sv, ids, gb, torch
        self.srcsets = [[int(x) for x in gg.sources(h, self.NSRC, seed=3)] for _, h, _ in graphs]
        self.free = {gi: list(range(self.POOL)) for gi in range(len(graphs))}
        self.bufs = {gi: [(torch.empty(h.n, dtype=torch.int32, device="cuda"),
                           torch.empty(h.n, dtype=torch.int32, device="cuda"))
                          for _ in range(self.POOL)] for gi, (_, h, _) in enumerate(graphs)}
        self.mult = {}
        self.digest_ref = {}
        self.full_ref = {}
        self.out = {}        # ticket -> (gi, kind, si, buf index)
        self.records = []    # per finished query: gi, kind, latency ms, retries, batch
        self.verified_full = 0
        self.verified_digest = 0
        self.pool_waits = 0

    def digest(self, gi, d, p):
        torch = self.torch
        if gi not in self.mult:
            n = d.numel()
            i = torch.arange(n, device="cuda", dtype=torch.int64)
            self.mult[gi] = ((i * 2654435761) % 2147483647 + 1, (i * 40503 + 12345) % 1000003 + 1)
        m1, m2 = self.mult[gi]
        dl = d.to(torch.int64) & 0xFFFFFFFF
        pl = p.to(torch.int64)
        return tuple(int(x) for x in torch.stack(
            [(dl * m1).sum(), (pl * m2).sum(), dl.sum(), pl.sum()]).cpu())

    def references(self):
        """Standalone results (gbgpu_bfs / gbgpu_wbfs) of every source a
        query can draw: digests, and full copies for the first two sources."""
        gb, torch = self.gb, self.torch
        for gi, (_, h, Gh) in enumerate(self.graphs):
            for kind in (0, 1):
                for si, s in enumerate(self.srcsets[gi]):
                    d, p = (gb.bfs if kind == 0 else gb.wbfs)(Gh, s)
                    self.digest_ref[(gi, kind, si)] = self.digest(gi, d, p)
                    if si < 2:
                        self.full_ref[(gi, kind, si)] = (d, p)
        torch.cuda.synchronize()

    def submit(self, gi, kind, si):
        while not self.free[gi]:
            self.pool_waits += 1
            self.harvest(block=True)
        b = self.free[gi].pop()
        d, p = self.bufs[gi][b]
        t = self.sv.submit(self.ids[gi], kind, self.srcsets[gi][si], d, p)
        self.out[t] = (gi, kind, si, b)

    def harvest(self, block=False):
        """Polls the outstanding tickets once (block: until one finished)."""
        while True:
            done = []
            for t in list(self.out):
                r = self.sv.poll(t)
                if r is not None:
                    done.append((t, r))
            for t, r in done:
                gi, kind, si, b = self.out.pop(t)
                assert r["status"] == 0, (self.graphs[gi][0], kind, r)
                d, p = self.bufs[gi][b]
                assert self.digest(gi, d, p) == self.digest_ref[(gi, kind, si)], \
                    f"served {self.graphs[gi][0]} kind {kind} src #{si} differs from standalone"
                self.verified_digest += 1
                if si < 2:
                    rd, rp = self.full_ref[(gi, kind, si)]
                    assert self.torch.equal(d, rd) and self.torch.equal(p, rp)
                    self.verified_full += 1
                self.records.append((gi, kind, (r["t_done_ns"] - r["t_arrive_ns"]) / 1e6,
                                     r["retries"], r["batch"], r["join_round"]))
                self.free[gi].append(b)
            if done or not block or not self.out:
                return
            time.sleep(0.0002)

    def finish(self):
        self.sv.drain()
        while self.out:
            self.harvest(block=True)

    def draw(self, rng):
        return (int(rng.integers(0, len(self.graphs))), int(rng.integers(0, 2)),
                int(rng.integers(0, self.NSRC)))

    def summary(self, records):
        lat = np.array([r[2] for r in records])
        out = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        per = {}
        for gi, (name, _, _) in enumerate(self.graphs):
            for kind, kname in ((0, "bfs"), (1, "wbfs")):
                sel = [r for r in records if r[0] == gi and r[1] == kind]
                if not sel:
                    continue
                l = np.array([r[2] for r in sel])
                per[f"{name}_{kname}"] = {
                    "n": len(sel), "p50_ms": round(float(np.percentile(l, 50)), 3),
                    "p99_ms": round(float(np.percentile(l, 99)), 3),
                    "retried": int(sum(1 for r in sel if r[3] > 0)),
                    "packed": int(sum(1 for r in sel if r[4] > 1)),
                    "joined": int(sum(1 for r in sel if r[5] > 0))}
        out["per_graph_kind"] = per
        return out


def run_serving(g, G, gg, gb, torch, nq=2000, cpu=True, workers=8):
    """Poisson arrivals of mixed BFS / weighted BFS queries on the six
    resident graphs, at 0.5x and 0.8x of the saturated rate, every served
    result verified against the standalone call."""
    # six resident graphs, weights uniform in [1, log2 n): RMAT scales 18,
    # 22, 24 and 26, the 256^3 torus, Erdos-Renyi 2^23 vertices of average
    # degree 32
    w24 = gg.weights(g, 24, seed=2)
    graphs = [("rmat24", g, gb.Graph(G.offsets, G.nbrs, w24, validate=False))]
    hosts = {"rmat24": (g, w24)}
    for name, make, W in (("rmat18", lambda: gg.rmat(18, seed=1), 18),
                          ("rmat22", lambda: gg.rmat(22, seed=1), 22),
                          ("rmat26", lambda: gg.rmat(26, seed=1), 26),
                          ("torus256", lambda: gg.torus3d(256), 24),
                          ("er23", lambda: gg.erdos_renyi(1 << 23, 32, seed=1), 23)):
        t = time.perf_counter()
        h = make().with_weights(W, seed=2)
        graphs.append((name, h, gb.Graph.from_csr(h, validate=False)))
        hosts[name] = (h, h.weights)
        log(f"serving graph {name}: n={h.n} m={h.m} loaded in {time.perf_counter() - t:.1f}s")
    # a weighted BFS on RMAT-26 takes ~9 GB of workspace (64 buckets of n/4)
    sv = gb.Server(arena_bytes=96 << 30, max_inflight=workers)
    ids = [sv.add_graph(GG) for _, _, GG in graphs]
    mix = ServedMix(graphs, sv, ids, gg, gb, torch)
    t = time.perf_counter()
    mix.references()
    log(f"serving: standalone references of {len(mix.digest_ref)} (graph, kind, source) in "
        f"{time.perf_counter() - t:.1f}s")
    rng = np.random.default_rng(7)

    # saturated throughput: the whole burst submitted at once (as far as the
    # output pools allow)
    def burst(count):
        t0 = time.perf_counter()
        for _ in range(count):
            mix.submit(*mix.draw(rng))
        mix.finish()
        return count / (time.perf_counter() - t0)
    burst(48)  # warm-up: every graph's workspaces and depth known
    mix.records.clear()
    w0 = mix.pool_waits
    qps_sat = burst(600)
    sat_records = list(mix.records)
    sat_waits = mix.pool_waits - w0

    # the same kind of mix one query at a time through gbgpu_bfs / gbgpu_wbfs
    def one_at_a_time(count):
        r2 = np.random.default_rng(7)
        t0 = time.perf_counter()
        for _ in range(count):
            gi, kind, si = mix.draw(r2)
            d, p = mix.bufs[gi][0]
            (gb.bfs if kind == 0 else gb.wbfs)(graphs[gi][2], mix.srcsets[gi][si], dist=d, parent=p)
        torch.cuda.synchronize()
        return count / (time.perf_counter() - t0)
    qps_single = one_at_a_time(300)
    log(f"serving: saturated {qps_sat:.1f} q/s, one at a time {qps_single:.1f} q/s")

    res = {"serving_saturated_qps": round(qps_sat, 1), "serving_single_qps": round(qps_single, 1),
           "serving_saturated": {**mix.summary(sat_records), "queries": 600,
                                 "pool_waits": sat_waits},
           "serving_graphs": "rmat18/22/24/26, torus256, er2^23 d32 (w < log2 n); 50/50 BFS/wBFS; "
                             "uniform graph; 32 seeded sources per graph"}
    for frac in (0.5, 0.8):
        lam = frac * qps_sat
        mix.records.clear()
        w0 = mix.pool_waits
        t0 = time.perf_counter()
        tnext = t0
        for _ in range(nq):
            tnext += rng.exponential(1.0 / lam)
            while time.perf_counter() < tnext:
                mix.harvest()
            mix.submit(*mix.draw(rng))
        mix.finish()
        el = time.perf_counter() - t0
        sm = mix.summary(mix.records)
        key = f"serving_lambda{int(frac * 10):02d}"
        # pool_waits: arrivals that found every output pair of their graph
        # in flight and waited for one (the arrival process then lags)
        res[key] = {"lambda_qps": round(lam, 1), "queries": nq, "qps": round(nq / el, 1), **sm,
                    "pool_waits": mix.pool_waits - w0}
        log(f"serving at {frac}x ({lam:.1f} q/s offered): {nq / el:.1f} q/s, p50 {sm['p50_ms']} "
            f"ms, p99 {sm['p99_ms']} ms")
        for k, v in sm["per_graph_kind"].items():
            log(f"    {k:16s} n={v['n']:4d} p50={v['p50_ms']:8.3f} p99={v['p99_ms']:8.3f} "
                f"retried={v['retried']} packed={v['packed']} joined={v['joined']}")
    res["serving_verified_digest"] = mix.verified_digest
    res["serving_verified_full"] = mix.verified_full
    sv.close()
    if not cpu:
        return res

    # the oracle on every host core: a seeded sample of the same mix, one
    # query per thread
    import oracle
    thr = min(16, len(os.sched_getaffinity(0)))
    r3 = np.random.default_rng(11)
    calls = []
    for _ in range(thr):
        gi, kind, si = mix.draw(r3)
        name = graphs[gi][0]
        h, w = hosts[name]
        s = mix.srcsets[gi][si]
        calls.append((lambda h=h, s=s: oracle.bfs(h, s)) if kind == 0 else
                     (lambda h=h, w=w, s=s: oracle.wbfs(h, s, weights=w)))
    qps, wall = oracle_all_cores(calls, thr)
    res["serving_oracle_all_cores_qps"] = round(qps, 3)
    res["serving_oracle_all_cores_threads"] = thr
    log(f"serving mix on the oracle, {thr} host threads: {qps:.3f} q/s ({wall:.1f} s)")
    return res


if __name__ == "__main__":
    main()
