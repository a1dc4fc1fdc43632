"""CPU tests of the server's scheduling policy (no GPU): the library's own group selection
and plan-cache eviction rules (phiks_server_select_group / _select_evictions, the
functions the server's worker and cache call), first case by case, then driving a
fake executor.  The fake server keeps the real server's state (pending queue in arrival
order, workspace arena, plan cache with reference counts and LRU ticks); it runs
admitted groups with injected latencies on a simulated clock and computes every
request with the CPU oracle, using the plan the host planner gives it.  Checked: every
request completes once and with the oracle's single-call result; each group is one
(p, n_scales) class and fits the arena; no request overtakes an earlier one of its
class; a plan held by an admitted request is never evicted; the cache stays within its
capacity except while every cached plan is in use (an out-of-memory condition injected
by a capacity smaller than one plan)."""
import heapq

import numpy as np
import pytest

import workloads
from oracle import phiks as ophiks

ph = pytest.importorskip("paper_2210_07667_amd")


def even(x):
    return (x + 1) & ~1


def test_group_takes_the_first_class_in_order():
    p = [2, 3, 2, 2, 3, 2]
    ns = [1, 1, 1, 2, 1, 1]
    ws = [10, 10, 10, 10, 10, 10]
    assert ph.server_select_group(p, ns, ws, 1000, 8) == [0, 2, 5]   # class (2, 1) only


def test_group_stops_at_the_first_request_that_does_not_fit():
    # request 2 would fit only if request 1 were skipped: it must not overtake it
    assert ph.server_select_group([1, 1, 1], [1, 1, 1], [30, 60, 10], 80, 8) == [0]
    # workspaces are rounded up to even doubles: 21 + 21 -> 22 + 22 = 44 > 43
    assert ph.server_select_group([1, 1], [1, 1], [21, 21], 43, 8) == [0]
    assert ph.server_select_group([1, 1], [1, 1], [21, 21], 44, 8) == [0, 1]


def test_group_size_limit_and_empty_queue():
    assert ph.server_select_group([1] * 10, [1] * 10, [2] * 10, 10 ** 6, 4) == [0, 1, 2, 3]
    assert ph.server_select_group([], [], [], 100, 4) == []
    # a first request larger than the arena alone is never admitted (submit refuses it)
    assert ph.server_select_group([1, 1], [1, 1], [101, 2], 100, 4) == []


def test_group_rejects_bad_arguments():
    with pytest.raises(RuntimeError):
        ph.server_select_group([1], [1], [2], 100, 0)


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

    def __init__(self, arena_doubles, max_group, capacity, rng):
        self.arena, self.max_group, self.capacity = arena_doubles, max_group, capacity
        self.rng = rng
        self.pending = []          # requests in arrival order
        self.cache = {}            # key -> dict(bytes, refs, last_use, plan)
        self.cache_bytes = 0
        self.tick = 0
        self.over_budget_with_free_entries = False
        self.groups = []

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

    def next_group(self):
        pick = ph.server_select_group([r["p"] for r in self.pending], [r["ns"] for r in self.pending],
                                      [r["ws"] for r in self.pending], self.arena, self.max_group)
        group = [self.pending[i] for i in pick]
        self.pending = [r for i, r in enumerate(self.pending) if i not in set(pick)]
        return group


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


@pytest.mark.parametrize("capacity_plans,max_group", [(3, 4), (0.5, 3), (100, 8)])
def test_fake_executor_runs_every_request_in_order_with_oracle_results(capacity_plans, max_group):
    rng = np.random.default_rng(17)
    reqs = _requests(rng, 40)
    unit = _plan_bytes([6, 5], 6, 11)
    server = FakeServer(arena_doubles=4 * max(r["ws"] for r in reqs), max_group=max_group,
                        capacity=int(capacity_plans * unit), rng=rng)
    arrivals = list(reqs)
    clock = 0.0
    done = {}
    inflight = []   # (finish time, seq, group)
    seq = 0
    while arrivals or server.pending or inflight:
        # arrivals up to the clock join the queue in order
        while arrivals and arrivals[0]["t"] <= clock:
            server.pending.append(arrivals.pop(0))
        if server.pending and len(inflight) < 2:
            group = server.next_group()
            assert group, "a non-empty queue must yield a group"
            assert len({(r["p"], r["ns"]) for r in group}) == 1
            assert sum(even(r["ws"]) for r in group) <= server.arena
            assert len(group) <= max_group
            for r in group:
                r["plan"] = server.plan(r)
            latency = float(rng.uniform(0.2, 3.0))          # injected executor latency
            heapq.heappush(inflight, (clock + latency, seq, group))
            seq += 1
            server.groups.append([r["id"] for r in group])
            continue
        # advance the clock to the next event
        nxt = [arrivals[0]["t"]] if arrivals else []
        if inflight:
            nxt.append(inflight[0][0])
        clock = max(clock, min(nxt))
        while inflight and inflight[0][0] <= clock:
            _, _, group = heapq.heappop(inflight)
            for r in group:
                s, q = r["plan"]["plan"]
                out = ophiks.phi_same_vector(r["A"], r["tau"], r["v"], r["p"], r["ns"], s, q)
                assert r["id"] not in done
                done[r["id"]] = (clock, out)
                r["plan"]["refs"] -= 1
    assert sorted(done) == [r["id"] for r in reqs]
    # no overtaking within a class: groups take each class's requests in arrival order
    order = [i for g in server.groups for i in g]
    for cls in {(r["p"], r["ns"]) for r in reqs}:
        ids = [i for i in order if (reqs[i]["p"], reqs[i]["ns"]) == cls]
        assert ids == sorted(ids)
    assert not server.over_budget_with_free_entries
    assert all(e["refs"] == 0 for e in server.cache.values())
    # every result is the oracle's single call for that request with its planned (s, q)
    for r in reqs[:8]:
        s, q, _ = ph.phiks_plan_params(r["A"], r["tau"], r["p"], r["ns"], r["tol"], "same_vector")
        ref = ophiks.phi_same_vector(r["A"], r["tau"], r["v"], r["p"], r["ns"], s, q)
        assert np.array_equal(done[r["id"]][1], ref)
