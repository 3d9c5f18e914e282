"""Definition-level checks for BFS / weighted-BFS outputs.

These verify a (dist, parent) pair against the problem statements directly
(Benchmark section, "Shortest Path Problems"), without running any search:

BFS (hop distances, int32, INT32_MAX = unreachable):
  * dist[src] == 0, parent[src] == src;
  * the reachable set is exactly src's connected component (scipy union of
    components, an independent routine);
  * |dist[u] - dist[v]| <= 1 on every edge inside the component;
  * every other reached v has parent[v] == min{u in N(v): dist[u] == dist[v]-1},
    which also proves dist[v] is achieved by a walk of that length;
  * unreachable vertices carry (INT32_MAX, -1).

Weighted BFS (uint32, 0xFFFFFFFF = unreachable):
  * dist[v] <= dist[u] + w(u,v) on every edge (no edge can shorten a path);
  * every reached v != src has a tight neighbour, and parent[v] is the
    smallest tight neighbour: dist[parent] + w == dist[v];
  * following parents strictly decreases dist, so the parent graph is a tree
    rooted at src (with positive weights, tightness alone implies this);
  * unreachable vertices carry (0xFFFFFFFF, -1).

Together the two weighted conditions characterise shortest-path distances
uniquely (a feasible potential that is tight along a tree from src equals the
distance function), so these checks pin the result without a second solver.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

BFS_INF = 2**31 - 1
WBFS_INF = 0xFFFFFFFF


def _sources_of_edges(g):
    return np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())


def component_mask(g, src):
    if g.m == 0:
        lab = np.arange(g.n)
    else:
        a = sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.nbrs, g.offsets), shape=(g.n, g.n))
        _, lab = connected_components(a, directed=False)
    return lab == lab[src]


def _min_over_lists(g, values, valid):
    """For each vertex v: min of values[e] over e in v's list with valid[e];
    INT64 max where none."""
    big = np.iinfo(np.int64).max
    vals = np.where(valid, values.astype(np.int64), big)
    out = np.full(g.n, big, dtype=np.int64)
    deg = g.degrees()
    nz = deg > 0
    if g.m:
        starts = g.offsets[:-1][nz]
        out[nz] = np.minimum.reduceat(vals, starts)
    return out


def check_bfs(g, src, dist, parent):
    """Raise AssertionError if (dist, parent) is not the BFS output."""
    dist = np.asarray(dist).astype(np.int64)
    parent = np.asarray(parent).astype(np.int64)
    n = g.n
    assert dist.shape == (n,) and parent.shape == (n,)
    assert dist[src] == 0, "dist[src] must be 0"
    assert parent[src] == src, "parent[src] must be src"
    comp = component_mask(g, src)
    reached = dist != BFS_INF
    assert np.array_equal(reached, comp), "reachable set differs from src's component"
    assert np.all(parent[~reached] == -1), "unreachable vertices must have parent -1"
    assert np.all(dist[reached] >= 0)
    u = _sources_of_edges(g)
    v = g.nbrs.astype(np.int64)
    inside = reached[u]
    assert np.all(np.abs(dist[u[inside]] - dist[v[inside]]) <= 1), "edge spans > 1 level"
    # minimum neighbour one level closer
    tight = reached[v] & reached[u] & (dist[v] == dist[u] - 1)
    best = _min_over_lists(g, v, tight)
    others = reached.copy()
    others[src] = False
    assert np.all(best[others] != np.iinfo(np.int64).max), "reached vertex without a closer neighbour"
    assert np.array_equal(parent[others], best[others]), "parent is not the min-ID closer neighbour"


def check_wbfs(g, src, dist, parent, weights=None):
    """Raise AssertionError if (dist, parent) is not the weighted-BFS output."""
    w = (g.weights if weights is None else weights).astype(np.int64)
    dist = np.asarray(dist).astype(np.uint64).astype(np.int64)
    parent = np.asarray(parent).astype(np.int64)
    n = g.n
    assert dist[src] == 0 and parent[src] == src
    reached = dist != WBFS_INF
    comp = component_mask(g, src)
    assert np.array_equal(reached, comp), "reachable set differs from src's component"
    assert np.all(parent[~reached] == -1)
    u = _sources_of_edges(g)
    v = g.nbrs.astype(np.int64)
    inside = reached[u]
    # feasibility: dist[v] <= dist[u] + w(u,v)   (edge stored in v's list: (v, u))
    assert np.all(dist[u[inside]] <= dist[v[inside]] + w[inside]), "edge violates the triangle inequality"
    tight = reached[u] & reached[v] & (dist[v] + w == dist[u])
    best = _min_over_lists(g, v, tight)
    others = reached.copy()
    others[src] = False
    assert np.all(best[others] != np.iinfo(np.int64).max), "reached vertex without a tight neighbour"
    assert np.array_equal(parent[others], best[others]), "parent is not the min-ID tight neighbour"
    # tree: parent distances strictly smaller (weights >= 1)
    p = parent[others]
    assert np.all(dist[p] < dist[others])
