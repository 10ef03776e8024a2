"""Admission scheduler (host-only native code) on a fake clock and a fake
device memory: the budget is never exceeded, requests start in arrival order
(no starvation), and a request larger than the budget is rejected."""

import numpy as np
import pytest

rmm = pytest.importorskip("paper_1505_07570_amd")


def test_fifo_budget_and_rejection():
    s = rmm.Scheduler(100)
    for rid, nb in [(1, 60), (2, 50), (3, 10), (4, 30)]:
        s.submit(rid, nb)
    assert s.admit() == [1]                  # 2 does not fit next to 1 ...
    assert s.stats() == {"in_use": 60, "queued": 3, "running": 1}
    s.complete(1)
    assert s.admit() == [2, 3, 4]            # ... and is not overtaken by 3 and 4
    with pytest.raises(rmm.RmmError):
        s.submit(5, 101)                     # can never run
    with pytest.raises(rmm.RmmError):
        s.submit(2, 1)                       # duplicate id
    with pytest.raises(rmm.RmmError):
        s.complete(99)                       # not running
    for rid in (2, 3, 4):
        s.complete(rid)
    assert s.stats() == {"in_use": 0, "queued": 0, "running": 0}


def test_simulated_serving_invariants():
    """Discrete-event run: random sizes, arrivals and service times."""
    rng = np.random.default_rng(7)
    budget = 1000
    s = rmm.Scheduler(budget)
    n = 400
    sizes = rng.integers(1, budget + 1, n)
    arrivals = np.cumsum(rng.exponential(1.0, n))
    service = rng.exponential(3.0, n)
    running = {}                             # id -> finish time
    started, t, nxt = [], 0.0, 0
    while nxt < n or running or s.stats()["queued"]:
        # next event: an arrival or a completion
        t_arr = arrivals[nxt] if nxt < n else np.inf
        t_fin = min(running.values()) if running else np.inf
        t = min(t_arr, t_fin)
        if t == t_fin:
            rid = min(running, key=running.get)
            del running[rid]
            s.complete(rid)
        else:
            s.submit(nxt, int(sizes[nxt]))
            nxt += 1
        for rid in s.admit():
            running[rid] = t + service[rid]
            started.append(rid)
        assert s.stats()["in_use"] == sum(int(sizes[r]) for r in running) <= budget
    assert started == list(range(n))         # first come, first served; nobody starves
