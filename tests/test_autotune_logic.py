"""Host logic of the autotuner (CPU): coordinate descent finds the best
configuration, never accepts a rejected candidate, and honours its budget."""
import json

from paper_1805_05208_amd import autotune


def test_descent_finds_separable_minimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30]}

    def cost(o):
        return (o["a"] - 3) ** 2 + (o["b"] - 20) ** 2 / 100.0 + 1.0

    r = autotune.coordinate_descent(space, {"a": 1, "b": 30}, cost, passes=3, budget_s=10)
    assert r["opts"] == {"a": 3, "b": 20}


def test_descent_never_accepts_rejected_candidates():
    space = {"a": [1, 2, 3, 4]}

    def cost(o):
        return None if o["a"] == 4 else 10.0 - o["a"]  # a=4 would be fastest but is "wrong"

    r = autotune.coordinate_descent(space, {"a": 1}, cost, passes=2, budget_s=10)
    assert r["opts"] == {"a": 3}
    assert {"a": 4} in r["rejected"]


def test_descent_budget_and_signature(tmp_path):
    calls = []

    def cost(o):
        calls.append(o)
        return 1.0

    r = autotune.coordinate_descent({"a": list(range(100))}, {"a": 0}, cost, budget_s=0.0)
    assert r["timed_out"] and len(calls) <= 2
    sig = autotune.signature(65536, 1819112, 9668, 7)
    assert sig == "n65536-m1819112-dmax2^13-low"
    path = tmp_path / "tuned.json"
    autotune.save([{"signature": sig, "kind": "bfs", "opts": {"tau": 10}, "cost": 0.1}], str(path))
    assert autotune.lookup(str(path), sig, "bfs") == {"tau": 10}
    assert autotune.lookup(str(path), sig, "wbfs") is None
    assert json.load(open(path))[sig]["bfs"]["seconds"] == 0.1


def test_small_graphs_try_small_grids():
    from paper_1805_05208_amd import autotune
    assert autotune.bfs_space(1 << 16)["grid"][:3] == [8, 16, 32]
    assert autotune.bfs_space(1 << 24)["grid"] == autotune.GRID_WIDE
    assert 20 in autotune.bfs_space(1 << 16)["tau"]


def test_search_never_ends_slower_than_its_start():
    from paper_1805_05208_amd import autotune
    costs = {5: 3.0, 10: 1.0, 20: 2.0}
    r = autotune.coordinate_descent({"tau": [5, 10, 20]}, {"tau": 20},
                                    lambda o: costs[o["tau"]], passes=2, budget_s=10)
    assert r["opts"] == {"tau": 10} and r["cost"] == 1.0 and r["start_cost"] == 2.0
    r = autotune.coordinate_descent({"tau": [5]}, {"tau": 20}, lambda o: costs[o["tau"]])
    assert r["opts"] == {"tau": 20} and r["cost"] == r["start_cost"] == 2.0
