"""Autotuner for the traversal knobs (direction threshold, dense-scan light
length, push chunk size, grid size, launches per completion check, bucket
window).

None of the knobs changes results, so the tuner treats them purely as speed
parameters, but it still re-checks that every candidate reproduces the
default configuration's outputs bit for bit before accepting its time.  The
search is coordinate descent (one knob at a time, repeated passes) under a
time budget.  Results are stored in a JSON file keyed by a graph signature
(vertices, stored edges, log2 of the maximum degree, diameter class from the
round count of the default run).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

GRID_WIDE = [64, 128, 256, 384, 512]
BFS_SPACE = {
    "tau": [5, 10, 20, 40, 80],
    "pull_light": [4, 8, 16, 32, 64],
    "wave_chunk": [64, 128, 256],
    "grid": GRID_WIDE,
    "rounds_per_sync": [1, 2, 3, 4, 6],
    "beta": [-1, 8, 24, 64],
}


def bfs_space(n: int) -> Dict[str, Sequence[int]]:
    """The BFS space for a graph of n vertices: on small graphs (at most 2^18
    vertices) a launch of hundreds of workgroups is mostly dispatch, so the
    grid also tries 8 to 32 workgroups."""
    sp = dict(BFS_SPACE)
    if n <= (1 << 18):
        sp["grid"] = [8, 16, 32] + GRID_WIDE
    return sp


WBFS_SPACE = {
    "tau": [5, 7, 10, 14, 20],
    "wave_chunk": [64, 128, 256],
    "grid": GRID_WIDE,
    "rounds_per_sync": [2, 3, 4, 8],
    "bucket_window": [0, 128, 256],
}


def wbfs_space(n: int) -> Dict[str, Sequence[int]]:
    """The weighted-BFS space for a graph of n vertices: bucket capacities
    from n/32 to n/2 entries (0 = the library's n/4, doubled and re-run on
    overflow), so the tuner can pick one that never overflows."""
    sp = dict(WBFS_SPACE)
    sp["bucket_capacity"] = [0] + [max(4096, n // d) for d in (32, 16, 8, 2)]
    return sp
MULTI_SPACE = {
    "tau": [5, 10, 20, 40],
    "wave_chunk": [64, 128, 256],
    "grid": [256, 384, 512],
}
DEFAULTS = {"tau": 20, "pull_light": 32, "wave_chunk": 256, "grid": 512, "rounds_per_sync": 3,
            "beta": 24}


def coordinate_descent(space: Dict[str, Sequence[int]], start: Dict[str, int],
                       cost: Callable[[Dict[str, int]], Optional[float]], passes: int = 2,
                       budget_s: float = 60.0, verbose: bool = False) -> Dict:
    """Minimise cost(opts) one knob at a time.  cost returns None for a
    rejected candidate (e.g. outputs differ).  Pure host logic."""
    t0 = time.time()
    best = dict(start)
    best_cost = cost(best)
    if best_cost is None:
        raise RuntimeError("the starting configuration was rejected")
    start_cost = best_cost
    tried = {tuple(sorted(best.items())): best_cost}
    rejected = []
    for _ in range(passes):
        improved = False
        for knob, values in space.items():
            for val in values:
                if time.time() - t0 > budget_s:
                    return {"opts": best, "cost": best_cost, "start_cost": start_cost,
                            "tried": len(tried), "rejected": rejected, "timed_out": True}
                cand = dict(best)
                cand[knob] = val
                key = tuple(sorted(cand.items()))
                if key in tried:
                    continue
                c = cost(cand)
                tried[key] = c
                if verbose:
                    print(f"  {knob}={val}: " + ("rejected" if c is None else f"{c * 1e3:.3f} ms")
                          + f" (best {best_cost * 1e3:.3f} ms)", flush=True)
                if c is None:
                    rejected.append(cand)
                    continue
                if c < best_cost * 0.98:
                    best, best_cost, improved = cand, c, True
        if not improved:
            break
    return {"opts": best, "cost": best_cost, "start_cost": start_cost, "tried": len(tried),
            "rejected": rejected, "timed_out": False}


def signature(n: int, m: int, max_degree: int, rounds: int) -> str:
    dclass = "low" if rounds < 16 else ("mid" if rounds < 256 else "high")
    return f"n{n}-m{m}-dmax2^{int(math.log2(max(max_degree, 1)))}-{dclass}"


def _median_time(fn, reps: int) -> float:
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def tune_bfs(G, srcs: List[int], reps: int = 3, budget_s: float = 60.0, passes: int = 2,
             space=None, verbose: bool = False) -> Dict:
    """Tune gbgpu_bfs on graph G for the given sources."""
    import torch
    import paper_1805_05208_amd as gb
    ref = [gb.bfs(G, s) for s in srcs]
    _, _, st = gb.bfs(G, srcs[0], stats=True)
    max_degree = int((G.offsets[1:] - G.offsets[:-1]).max().item())

    def cost(opts):
        for s, (d0, p0) in zip(srcs, ref):
            d, p = gb.bfs(G, s, opts=opts)
            if not (torch.equal(d, d0) and torch.equal(p, p0)):
                return None
        return _median_time(lambda: [gb.bfs(G, s, opts=opts) for s in srcs], reps)

    res = coordinate_descent(space or bfs_space(G.n), dict(DEFAULTS), cost, passes, budget_s, verbose)
    res["default_cost"] = cost(dict(DEFAULTS))
    res["signature"] = signature(G.n, G.m, max_degree, st["rounds"])
    res["kind"] = "bfs"
    return res


def tune_wbfs(G, srcs: List[int], reps: int = 2, budget_s: float = 60.0, passes: int = 2,
              space=None, verbose: bool = False) -> Dict:
    import torch
    import paper_1805_05208_amd as gb
    ref = [gb.wbfs(G, s) for s in srcs]
    _, _, st = gb.wbfs(G, srcs[0], stats=True)
    max_degree = int((G.offsets[1:] - G.offsets[:-1]).max().item())
    start = {"tau": 10, "wave_chunk": 256, "grid": 512, "rounds_per_sync": 3,
             "bucket_window": 0, "bucket_capacity": 0}

    def cost(opts):
        for s, (d0, p0) in zip(srcs, ref):
            # (a capacity that overflows re-runs the search, which the
            # timing below includes)
            d, p = gb.wbfs(G, s, opts=opts)
            if not (torch.equal(d, d0) and torch.equal(p, p0)):
                return None
        return _median_time(lambda: [gb.wbfs(G, s, opts=opts) for s in srcs], reps)

    res = coordinate_descent(space or wbfs_space(G.n), start, cost, passes, budget_s, verbose)
    res["default_cost"] = cost(start)
    res["signature"] = signature(G.n, G.m, max_degree, st["rounds"])
    res["kind"] = "wbfs"
    return res


def tune_multi(G, srcs: List[int], reps: int = 2, budget_s: float = 60.0, passes: int = 1,
               space=None, verbose: bool = False) -> Dict:
    import torch
    import paper_1805_05208_amd as gb
    D0, P0 = gb.bfs_multi(G, srcs)
    max_degree = int((G.offsets[1:] - G.offsets[:-1]).max().item())
    start = {"tau": 20, "wave_chunk": 256, "grid": 512}

    def cost(opts):
        D, P = gb.bfs_multi(G, srcs, opts=opts)
        if not (torch.equal(D, D0) and torch.equal(P, P0)):
            return None
        return _median_time(lambda: gb.bfs_multi(G, srcs, opts=opts), reps)

    res = coordinate_descent(space or MULTI_SPACE, start, cost, passes, budget_s, verbose)
    res["default_cost"] = cost(start)
    res["signature"] = signature(G.n, G.m, max_degree, 0)
    res["kind"] = "multi"
    return res


def save(results: Sequence[Dict], path: str) -> None:
    db = {}
    if os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
    for r in results:
        db.setdefault(r["signature"], {})[r["kind"]] = {
            "opts": r["opts"], "seconds": r["cost"], "default_seconds": r.get("default_cost")}
    with open(path, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)


def lookup(path: str, sig: str, kind: str) -> Optional[Dict[str, int]]:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        db = json.load(f)
    return db.get(sig, {}).get(kind, {}).get("opts")


def main():
    """python -m paper_1805_05208_amd.autotune [--graph rmat|torus] --scale 24 [--budget 120]"""
    import argparse
    import torch
    import graphgen as gg
    import paper_1805_05208_amd as gb
    ap = argparse.ArgumentParser()
    ap.add_argument("--graph", choices=["rmat", "torus"], default="rmat")
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--sources", type=int, default=8)
    ap.add_argument("--budget", type=float, default=120.0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tuned.json"))
    ap.add_argument("--kinds", default="bfs,wbfs,multi")
    args = ap.parse_args()
    if args.graph == "torus":
        g = gg.torus3d(round(2 ** (args.scale / 3)))
    else:
        g = gg.rmat(args.scale, seed=1)
    w = gg.weights(g, max(2, int(math.log2(g.n))), seed=2)
    G = gb.Graph(g.offsets, g.nbrs, w, validate=False)
    srcs = [int(s) for s in gg.sources(g, args.sources, seed=3)]
    results = []
    kinds = args.kinds.split(",")
    if "bfs" in kinds:
        results.append(tune_bfs(G, srcs, budget_s=args.budget, verbose=True))
        print("bfs", results[-1]["opts"], results[-1]["cost"], results[-1]["default_cost"], flush=True)
    if "wbfs" in kinds:
        results.append(tune_wbfs(G, srcs[:2], budget_s=args.budget, verbose=True))
        print("wbfs", results[-1]["opts"], results[-1]["cost"], results[-1]["default_cost"], flush=True)
    if "multi" in kinds:
        s64 = [int(s) for s in gg.sources(g, 64, seed=3)]
        results.append(tune_multi(G, s64, budget_s=args.budget, verbose=True))
        print("multi", results[-1]["opts"], results[-1]["cost"], results[-1]["default_cost"], flush=True)
    save(results, args.out)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
