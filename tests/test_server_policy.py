"""CPU tests of the server's policy (no GPU): the library's lane routing and plan-cache
eviction rules (phiks_server_lane / _select_evictions, the functions the server's
admission and cache call), case by case, and a fake executor driving the eviction rule
with the oracle computing every request.  The serving engine's threads, admission and
workspace slots are checked by tests/host/server_core_check.cpp under the thread and
address sanitizers (test_host_sanitize.py).  Fake executor: requests arrive in order,
each is planned by the host planner through the cache (reference counts, LRU ticks),
runs for an injected latency on a simulated clock with at most a few running at once,
and is computed with the CPU oracle.  Checked: every request completes once and with
the oracle's single-call result; a plan held by a running request is never evicted;
the cache stays within its capacity except while every cached plan is in use (an
out-of-memory condition injected by a capacity smaller than one plan)."""
import heapq

import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

ph = pytest.importorskip("paper_2210_07667_amd")


def even(x):
    return (x + 1) & ~1


def test_lanes_by_size():
    """Lane 0 up to 2^18 values, then one lane per factor 8, capped at lanes - 1."""
    assert ph.server_lane(1, 3) == 0
    assert ph.server_lane(256 * 256, 3) == 0
    assert ph.server_lane(64 ** 3, 3) == 0            # 2^18
    assert ph.server_lane(64 ** 3 + 1, 3) == 1
    assert ph.server_lane(1024 * 1024, 3) == 1        # 2^20
    assert ph.server_lane(128 ** 3, 3) == 1           # 2^21
    assert ph.server_lane(192 ** 3, 3) == 2
    assert ph.server_lane(256 ** 3, 3) == 2
    assert ph.server_lane(256 ** 3, 4) == 2
    assert ph.server_lane(1 << 30, 4) == 3
    assert ph.server_lane(1 << 30, 1) == 0
    with pytest.raises(ph.PhiksError):
        ph.server_lane(0, 3)
    with pytest.raises(ph.PhiksError):
        ph.server_lane(10, 0)


def test_evictions_least_recently_used_unreferenced_first():
    nbytes = [100, 200, 300, 400]
    refs = [0, 1, 0, 0]
    last = [5, 1, 9, 2]
    # 1000 held, 350 incoming, room 900: evict 400 (tick 2) -> 600 + 350 fits? 950 > 900,
    # then 100 (tick 5) -> 500 + 350 = 850 fits
    assert ph.server_select_evictions(nbytes, refs, last, 1000, 350, 900) == [3, 0]
    # enough room: nothing evicted
    assert ph.server_select_evictions(nbytes, refs, last, 1000, 350, 2000) == []
    # every entry in use: nothing evicted, the cache runs over budget
    assert ph.server_select_evictions(nbytes, [1, 1, 1, 1], last, 1000, 350, 500) == []
    # only unreferenced entries go, even when the new plan still does not fit
    assert ph.server_select_evictions(nbytes, refs, last, 1000, 350, 100) == [3, 0, 2]


def _plan_bytes(n, s, q):
    # device matrices of one plan: (q - 1) node matrices and s + 1 squaring levels per mode
    return sum((q - 1 + s + 1) * m * m * 8 for m in n)


class FakeServer:
    """The server's state and decisions on a simulated clock; the executor is the oracle."""

    def __init__(self, capacity, rng):
        self.capacity = capacity
        self.rng = rng
        self.cache = {}            # key -> dict(bytes, refs, last_use, plan)
        self.cache_bytes = 0
        self.tick = 0
        self.over_budget_with_free_entries = False

    def plan(self, r):
        key = (r["op"], r["tau"], r["p"], r["ns"])
        self.tick += 1
        if key in self.cache:
            e = self.cache[key]
            e["refs"] += 1
            e["last_use"] = self.tick
            return e
        s, q, _ = ph.phiks_plan_params(r["A"], r["tau"], r["p"], r["ns"], r["tol"], "same_vector")
        nb = _plan_bytes(r["n"], s, q)
        keys = list(self.cache)
        victims = ph.server_select_evictions([self.cache[k]["bytes"] for k in keys],
                                             [self.cache[k]["refs"] for k in keys],
                                             [self.cache[k]["last_use"] for k in keys],
                                             self.cache_bytes, nb, self.capacity)
        for i in victims:
            assert self.cache[keys[i]]["refs"] == 0, "an admitted request's plan was evicted"
            self.cache_bytes -= self.cache[keys[i]]["bytes"]
            del self.cache[keys[i]]
        e = {"bytes": nb, "refs": 1, "last_use": self.tick, "plan": (s, q)}
        self.cache[key] = e
        self.cache_bytes += nb
        if self.cache_bytes > self.capacity and any(x["refs"] == 0 for x in self.cache.values()):
            self.over_budget_with_free_entries = True
        return e


def _requests(rng, count):
    shapes = [[6, 5], [4, 3, 5], [7], [5, 6]]
    ops = [[workloads.adr_1d(m, 0.5, 1.0 / (j + 1), -1.0) for j, m in enumerate(n)] for n in shapes]
    reqs = []
    t = 0.0
    for i in range(count):
        t += rng.exponential(1.0)
        k = int(rng.integers(len(shapes)))
        n = shapes[k]
        p = int(rng.integers(1, 3))
        ns = int(rng.integers(1, 3))
        tau = float(rng.choice([1e-2, 3e-2]))
        N = int(np.prod(n))
        t_ = max(11, p, 1)
        reqs.append({"id": i, "t": t, "op": k, "n": n, "A": ops[k], "p": p, "ns": ns, "tau": tau,
                     "tol": 2.0 ** -53, "v": workloads.randn_vec(n, 1000 + i),
                     "ws": (2 * t_ + 2 * p) * N})
    return reqs


@pytest.mark.parametrize("capacity_plans,running", [(3, 4), (0.5, 3), (100, 8)])
def test_fake_executor_runs_every_request_with_oracle_results(capacity_plans, running):
    rng = np.random.default_rng(17)
    reqs = _requests(rng, 40)
    unit = _plan_bytes([6, 5], 6, 11)
    server = FakeServer(capacity=int(capacity_plans * unit), rng=rng)
    arrivals = list(reqs)
    queue = []
    clock = 0.0
    done = {}
    inflight = []   # (finish time, seq, request)
    seq = 0
    while arrivals or queue or inflight:
        while arrivals and arrivals[0]["t"] <= clock:
            queue.append(arrivals.pop(0))
        if queue and len(inflight) < running:
            r = queue.pop(0)                                  # admission in arrival order
            r["plan"] = server.plan(r)
            latency = float(rng.uniform(0.2, 3.0))            # injected executor latency
            heapq.heappush(inflight, (clock + latency, seq, r))
            seq += 1
            continue
        nxt = [arrivals[0]["t"]] if arrivals else []
        if inflight:
            nxt.append(inflight[0][0])
        clock = max(clock, min(nxt))
        while inflight and inflight[0][0] <= clock:
            _, _, r = heapq.heappop(inflight)
            s, q = r["plan"]["plan"]
            out = ophiks.phi_same_vector(r["A"], r["tau"], r["v"], r["p"], r["ns"], s, q)
            assert r["id"] not in done
            done[r["id"]] = (clock, out)
            r["plan"]["refs"] -= 1
    assert sorted(done) == [r["id"] for r in reqs]
    assert not server.over_budget_with_free_entries
    assert all(e["refs"] == 0 for e in server.cache.values())
    # every result is the oracle's single call for that request with its planned (s, q)
    for r in reqs[:8]:
        s, q, _ = ph.phiks_plan_params(r["A"], r["tau"], r["p"], r["ns"], r["tol"], "same_vector")
        ref = ophiks.phi_same_vector(r["A"], r["tau"], r["v"], r["p"], r["ns"], s, q)
        assert np.array_equal(done[r["id"]][1], ref)
