"""Scheduling logic of the continuous-batching server, on the CPU with a fake batch that
models slots, an HBM budget and per-step cost (no GPU; the device batch is tested in
test_gpu_batch.py / test_gpu_serve.py)."""
import types

import numpy as np
import pytest

import workloads
from paper_2212_14153_amd import serve

DONE = 1


class FakeBatch:
    """Slots + budget admission; run(k) advances every member by min(k, remaining) and
    charges time on a virtual clock proportional to the nodes advanced."""

    def __init__(self, slots, budget, clock, ns_per_node_step=1e-9):
        self.slots, self.budget, self.clock = slots, budget, clock
        self.cost = ns_per_node_step
        self.members = {}
        self.next = 1
        self.max_concurrent = 0
        self.max_used = 0
        self.finished = []

    def set_launch(self, cfg):
        pass

    def close(self):
        pass

    def used(self):
        return sum(m["bytes"] for m in self.members.values())

    def try_add(self, params, R, steps):
        need = params.nodes * 36
        if len(self.members) >= self.slots or self.used() + need > self.budget:
            return None
        sid = self.next
        self.next += 1
        self.members[sid] = {"nodes": params.nodes, "left": steps, "bytes": need,
                             "R": np.asarray(R) + steps, "reported": False}
        self.max_concurrent = max(self.max_concurrent, len(self.members))
        self.max_used = max(self.max_used, self.used())
        return sid

    def run(self, k):
        act = [m for m in self.members.values() if m["left"] > 0]
        if not act:
            return 0
        s = min(k, min(m["left"] for m in act))
        self.clock.t += s * sum(m["nodes"] for m in act) * self.cost
        for m in act:
            m["left"] -= s
        return s

    def launch(self, k):   # the device batch's asynchronous half; wait() completes it
        return self.run(k)

    def wait(self):
        pass

    def poll(self):
        out = []
        for sid, m in self.members.items():
            if m["left"] == 0 and not m["reported"]:
                m["reported"] = True
                out.append((sid, DONE))
        return out

    def beads(self, sid):
        return self.members[sid]["R"], None, None

    def release(self, sid):
        del self.members[sid]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def make_requests(n, rate, seed=1, steps=1000):
    t = workloads.poisson_arrivals(n, rate=rate, seed=seed)
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        nodes = int(rng.integers(1000, 5000))
        p = types.SimpleNamespace(nodes=nodes, nx=nodes, ny=1)
        reqs.append(serve.Request(i, p, np.zeros((2, 2)), steps, float(t[i])))
    return reqs


def run_server(reqs, slots, budget, chunk=100, lanes=1):
    clock = Clock()
    fbs = [FakeBatch(slots, budget, clock) for _ in range(lanes)]
    fb = fbs[0] if lanes == 1 else fbs
    orig = serve._lib.FPD_SIM_DONE
    srv = serve.Server("f16dev", budget, slots, chunk=chunk, clock=clock, batch=fb)
    # the fake clock only moves when work runs: idle waits jump to the next arrival
    serve_time = serve.time

    class T:
        @staticmethod
        def sleep(dt):
            clock.t += max(dt, 1e-6)

        perf_counter = staticmethod(clock)

    serve.time = T
    try:
        done = srv.serve(reqs)
    finally:
        serve.time = serve_time
    assert orig == DONE
    return done, fb


def test_poisson_arrivals_rate_and_seed():
    t = workloads.poisson_arrivals(20000, rate=50.0, seed=50)
    assert np.all(np.diff(t) > 0)
    assert len(t) / t[-1] == pytest.approx(50.0, rel=0.03)
    assert np.array_equal(t, workloads.poisson_arrivals(20000, rate=50.0, seed=50))


def test_every_request_completes_with_its_own_result():
    reqs = make_requests(60, rate=5000.0)
    done, fb = run_server(reqs, slots=8, budget=10 ** 9)
    assert len(done) == 60 and all(r.status == DONE for r in done)
    for r in done:
        assert np.array_equal(r.beads, np.zeros((2, 2)) + r.steps)
        assert r.arrival <= r.admitted <= r.finished
    assert not fb.members                     # every slot was released
    assert fb.max_concurrent == 8             # slots were the binding limit


def test_budget_limits_concurrency_and_requests_overlap():
    reqs = make_requests(40, rate=1000.0, seed=3)
    budget = 3 * 5000 * 36                    # room for three of the largest at once
    done, fb = run_server(reqs, slots=64, budget=budget)
    assert fb.max_used <= budget
    assert fb.max_used > budget - 5000 * 36   # the budget, not the slots, was binding
    assert fb.max_concurrent >= 3             # several requests run together
    # FIFO admission: admission order follows arrival order
    adm = [r.rid for r in sorted(done, key=lambda r: r.admitted)]
    assert adm == sorted(adm)


def test_summary_percentiles_and_fifo_replay():
    reqs = make_requests(30, rate=100.0, seed=4)
    done, _ = run_server(reqs, slots=4, budget=10 ** 9)
    s = serve.summarize(done, warmup=5)
    lat = sorted(r.latency for r in sorted(done, key=lambda r: r.arrival)[5:])
    assert s["requests"] == 25 and s["completed"] == 25
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_s"] >= s["p50_s"]
    # single FIFO server: waiting accumulates when service exceeds the gaps
    lat_f = serve.fifo_replay([0.0, 0.1, 0.2], [0.5, 0.5, 0.5])
    assert np.allclose(lat_f, [0.5, 0.9, 1.3])


def test_run_batches_interleaves_launches_and_stops():
    """run_batches: every round enqueues each live batch before any wait, slices are
    bounded, a batch whose simulations are done (launch returns 0) drops out."""
    log = []

    class FakeBatch:
        def __init__(self, name, remaining):
            self.name, self.remaining, self.pending = name, remaining, False

        def launch(self, n):
            assert not self.pending
            adv = min(n, self.remaining)
            self.remaining -= adv
            self.pending = True
            log.append(("launch", self.name, adv))
            return adv

        def wait(self):
            self.pending = False
            log.append(("wait", self.name))

    a, b = FakeBatch("a", 1000), FakeBatch("b", 300)
    assert serve.run_batches([a, b], 700, slice_steps=256) == [700, 300]
    assert (a.remaining, b.remaining) == (300, 0)
    # first round: both launched, then both waited
    assert log[:4] == [("launch", "a", 256), ("launch", "b", 256), ("wait", "a"),
                       ("wait", "b")]
    assert max(n for kind, *rest in log if kind == "launch" for n in rest[1:]) <= 256
    assert not a.pending and not b.pending


def test_requests_spread_over_lanes():
    """Two batches (lanes): every request completes, each in one lane, both lanes take
    work, and the result is the request's own."""
    reqs = make_requests(40, rate=200.0, steps=500)
    done, fbs = run_server(reqs, slots=8, budget=1 << 40, chunk=100, lanes=2)
    assert sorted(r.rid for r in done) == list(range(40))
    assert {r.lane for r in done} == {0, 1}
    for r in done:
        assert r.status == DONE and np.array_equal(r.beads, np.zeros((2, 2)) + 500)
    assert all(not fb.members for fb in fbs)
