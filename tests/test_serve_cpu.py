"""Scheduling of the serving loop (admission, memory budget, slots, continuous batching,
failures, latency accounting) with a simulated executor and clock; no GPU."""
import numpy as np
import pytest

from paper_2107_01664_amd import serve


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeExecutor:
    """Each handle costs `bytes_per_face * nF`; a shared step costs a fixed overhead plus
    a term per mesh, so batching saves the overhead.  Records every call."""

    def __init__(self, clock, budget, overhead=1e-3, per_face=1e-7, bytes_per_face=1000,
                 fail=None):
        self.clock, self.budget = clock, budget
        self.overhead, self.per_face, self.bpf = overhead, per_face, bytes_per_face
        self.live = {}
        self.batches = []
        self.fail = fail or {}          # rid -> step index (1-based) that fails
        self.next = 0

    def estimate(self, req):
        return self.bpf * req.F.shape[0]

    def create(self, req):
        h = self.next
        self.next += 1
        self.live[h] = [req, 0]
        assert sum(self.estimate(r) for r, _ in self.live.values()) <= self.budget
        return h

    def step(self, handles):
        assert len(set(handles)) == len(handles)
        self.batches.append([self.live[h][0].rid for h in handles])
        cost = self.overhead
        sts, es = [], []
        for h in handles:
            req, k = self.live[h]
            self.live[h][1] = k + 1
            cost += self.per_face * req.F.shape[0]
            sts.append(4 if self.fail.get(req.rid) == k + 1 else 0)
            es.append(1.0 / (k + 1))
        self.clock.t += cost
        return sts, es

    def vertices(self, h):
        return self.live[h][0].V

    def destroy(self, h):
        del self.live[h]


def make_requests(n=20, seed=0, steps=4, rate=50.0):
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1 / rate, n))
    out = []
    for q in range(n):
        nF = int(rng.integers(1000, 20000))
        out.append(serve.Request(q, float(arr[q]), np.zeros((nF // 2, 3)), np.zeros((nF, 3), np.int32),
                                 steps))
    return out


def run_sim(reqs, budget=10**8, max_active=16, **kw):
    clk = SimClock()
    ex = FakeExecutor(clk, budget, **kw)
    res = serve.run(reqs, ex, budget, max_active, clock=clk, sleep=clk.sleep)
    return res, ex


def test_all_steps_done_and_ordered():
    reqs = make_requests()
    res, ex = run_sim(reqs)
    assert [r.rid for r in res] == list(range(len(reqs)))
    for r, q in zip(res, reqs):
        assert r.status == 0
        assert len(r.step_done) == q.steps
        assert r.admitted >= q.arrival
        assert np.all(np.diff(r.step_done) > 0)
        assert r.finished == r.step_done[-1]
    assert not ex.live
    # arrival order is admission order
    adm = [r.admitted for r in sorted(res, key=lambda r: (r.arrival, r.rid))]
    assert np.all(np.diff(adm) >= 0)


def test_memory_budget_and_slots_respected():
    reqs = make_requests(n=30, rate=1e6)              # everything arrives at once
    budget = 40000 * 1000                              # about three average meshes
    res, ex = run_sim(reqs, budget=budget, max_active=4)
    assert all(len(b) <= 4 for b in ex.batches)
    assert all(r.status == 0 for r in res)
    # the budget bound is asserted inside FakeExecutor.create; several meshes did share steps
    assert max(len(b) for b in ex.batches) >= 2


def test_request_larger_than_budget_is_rejected():
    reqs = make_requests(n=5, rate=1e6)
    big = max(reqs, key=lambda r: r.F.shape[0])
    budget = big.F.shape[0] * 1000 - 1
    res, ex = run_sim(reqs, budget=budget)
    r = [x for x in res if x.rid == big.rid][0]
    assert r.status == -1 and not r.step_done
    assert all(x.status == 0 for x in res if x.rid != big.rid)


def test_continuous_admission_joins_running_batch():
    # A long request is running when a short one arrives: the short one joins the next
    # round and leaves first, while the long one keeps stepping.
    V, F = np.zeros((10, 3)), np.zeros((20000, 3), np.int32)
    a = serve.Request(0, 0.0, V, F, steps=20)
    b = serve.Request(1, 0.005, V, F[:2000], steps=2)
    res, ex = run_sim([a, b], overhead=1e-3, per_face=1e-7)
    ra, rb = res
    assert rb.admitted < ra.finished
    assert rb.finished < ra.finished
    assert any(len(bt) == 2 for bt in ex.batches)
    assert rb.admitted - rb.arrival < 0.01            # waited at most about one round


def test_failure_retires_only_that_request():
    reqs = make_requests(n=6, rate=1e6)
    res, ex = run_sim(reqs, fail={2: 2})
    bad = [r for r in res if r.rid == 2][0]
    assert bad.status == 4 and len(bad.step_done) == 2
    assert all(r.status == 0 and len(r.step_done) == 4 for r in res if r.rid != 2)
    assert not ex.live


def test_serial_reference_has_no_overlap():
    reqs = make_requests(n=8)
    clk = SimClock()
    ex = FakeExecutor(clk, 10**9)
    res = serve.run_serial(reqs, ex, clock=clk, sleep=clk.sleep)
    order = sorted(res, key=lambda r: (r.arrival, r.rid))
    for p, q in zip(order, order[1:]):
        assert q.admitted >= p.finished
    assert all(len(b) == 1 for b in ex.batches)


def test_batching_beats_serial_under_load():
    reqs = make_requests(n=40, rate=1e6, steps=3)
    res, _ = run_sim(reqs, overhead=5e-3, per_face=1e-8)
    clk = SimClock()
    ser = serve.run_serial(reqs, FakeExecutor(clk, 10**9, overhead=5e-3, per_face=1e-8),
                           clock=clk, sleep=clk.sleep)
    a, b = serve.summary(res), serve.summary(ser)
    assert a["steps"] == b["steps"] == 120
    assert a["steps_per_s"] > 2 * b["steps_per_s"]
    assert a["request_latency_ms"]["p99"] < b["request_latency_ms"]["p99"]


def test_summary_latencies():
    reqs = make_requests(n=5, steps=3)
    res, _ = run_sim(reqs)
    s = serve.summary(res)
    lat = [x for r in res for x in r.step_latencies()]
    assert s["steps"] == 15
    assert s["step_latency_ms"]["p50"] == pytest.approx(np.percentile(np.array(lat) * 1e3, 50))
    assert all(x > 0 for x in lat)


def test_lanes_bound_small_request_latency():
    # two large meshes (long steps) and a stream of small ones: with lanes, a small mesh's
    # step waits for at most one large step; with a single lane it waits for all of them
    rng = np.random.default_rng(3)
    V = np.zeros((10, 3))
    big = [serve.Request(q, 0.0, V, np.zeros((200000, 3), np.int32), steps=6) for q in range(2)]
    small = [serve.Request(2 + q, 0.01 * q, V, np.zeros((int(rng.integers(2000, 8000)), 3), np.int32), steps=3)
             for q in range(12)]
    reqs = big + small
    lat = {}
    for policy in (None, 50000):
        clk = SimClock()
        ex = FakeExecutor(clk, 10**12, overhead=1e-3, per_face=1e-7)
        res = serve.run(reqs, ex, 10**12, 16, clock=clk, sleep=clk.sleep, small_faces=policy, max_large=2)
        assert all(r.status == 0 and len(r.step_done) == r_.steps for r, r_ in zip(res, reqs))
        assert not ex.live
        small_lat = [x for r in res if r.nF <= 50000 for x in r.step_latencies()]
        lat[policy] = max(small_lat)
        if policy is not None:
            # no shared step mixes lanes, and a large mesh always steps alone
            for b in ex.batches:
                assert all(r < 2 for r in b) or all(r >= 2 for r in b)
                assert len(b) == 1 or all(r >= 2 for r in b)
            # one large step (0.02 s) plus one small batch bounds a small step's latency
            assert lat[policy] < 0.02 + 0.001 + 12 * 8000 * 1e-7 + 1e-3 + 1e-9
    assert lat[50000] < lat[None]


def test_lanes_in_arrival_order():
    # lane_order "oldest": a large request that arrived first runs its steps back to back,
    # as on the serial path, while the small requests behind it wait and then share steps;
    # a small request that arrived before the large one goes first
    V = np.zeros((10, 3))
    first = serve.Request(0, 0.0, V, np.zeros((3000, 3), np.int32), steps=2)
    big = serve.Request(1, 0.001, V, np.zeros((200000, 3), np.int32), steps=4)
    small = [serve.Request(2 + q, 0.002 + 0.001 * q, V, np.zeros((4000, 3), np.int32), steps=2) for q in range(5)]
    clk = SimClock()
    ex = FakeExecutor(clk, 10**12)
    res = serve.run([first, big] + small, ex, budget_bytes=10**12, max_active=16, clock=clk, sleep=clk.sleep,
                    small_faces=50000, lane_order="oldest")
    by = {r.rid: r for r in res}
    assert all(r.status == 0 for r in res)
    # the large request's steps are consecutive batches of one
    big_rounds = [i for i, b in enumerate(ex.batches) if b == [1]]
    assert big_rounds == list(range(big_rounds[0], big_rounds[0] + 4))
    # the first small request is stepped before the large one starts
    assert by[0].step_done[0] < by[1].step_done[0]
    # the later small ones start after the large one is done and share their steps
    assert all(by[r].step_done[0] > by[1].finished for r in range(2, 7))
    assert any(len(b) >= 5 for b in ex.batches)
    with pytest.raises(ValueError):
        serve.run(small, ex, budget_bytes=10**12, small_faces=50000, lane_order="lifo")
