"""The serving scheduler on a host-only engine (no GPU): continuous batching
by (model, layer), FIFO admission under an HBM budget, every request
completes every layer exactly once."""
from paper_2409_07751_amd.serve import Request, Server, latency_report


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance_to(self, t):
        self.t = max(self.t, t)


class FakeEngine:
    """A layer of model m costs cost[m] seconds whatever the batch size; the
    'ciphertext' is the list of layers applied so far."""

    def __init__(self, clock, layers, cost, work):
        self.clock, self.layers, self.cost, self.work = clock, layers, cost, work
        self.calls = []
        self.peak_inflight = 0

    def n_layers(self, m):
        return self.layers[m]

    def run_layer(self, m, layer, cts):
        self.calls.append((m, layer, len(cts)))
        self.clock.t += self.cost[m]
        return [c + [(m, layer)] for c in cts]

    def sync(self):
        pass

    def working_bytes(self, m):
        return self.work[m]


def make(n, clock, models, spacing):
    return [Request(i, models[i % len(models)], [], arrival=i * spacing) for i in range(n)]


def test_every_request_runs_every_layer_once_and_batches_form():
    clock = FakeClock()
    eng = FakeEngine(clock, {"a": 3, "b": 2}, {"a": 1.0, "b": 1.0}, {"a": 10, "b": 10})
    reqs = make(20, clock, ["a", "b"], 0.1)
    srv = Server(eng, hbm_budget=1000, max_batch=8)
    done = srv.run(reqs, clock=clock)
    assert len(done) == 20
    for r in done:
        assert r.ct == [(r.model, i) for i in range(eng.layers[r.model])]
        assert r.done >= r.arrival
    # arrivals during a layer join a later batch of size > 1
    assert max(n for _, _, n in eng.calls) > 1
    assert all(n <= 8 for _, _, n in eng.calls)
    rep = latency_report(done)
    assert rep["requests"] == 20 and rep["latency_ms_p99"] >= rep["latency_ms_p50"]


def test_budget_limits_requests_in_flight():
    clock = FakeClock()
    eng = FakeEngine(clock, {"a": 2}, {"a": 1.0}, {"a": 100})
    reqs = make(10, clock, ["a"], 0.0)
    srv = Server(eng, hbm_budget=250, max_batch=16)
    orig = srv._step
    seen = []

    def step(now_fn):
        seen.append(len(srv.active))
        assert srv.in_use <= 250
        orig(now_fn)

    srv._step = step
    done = srv.run(reqs, clock=clock)
    assert len(done) == 10 and max(seen) == 2
    assert all(n <= 2 for _, _, n in eng.calls)


def test_single_request_bigger_than_budget_still_runs_alone():
    clock = FakeClock()
    eng = FakeEngine(clock, {"a": 1}, {"a": 1.0}, {"a": 500})
    done = Server(eng, hbm_budget=100).run(make(3, clock, ["a"], 0.0), clock=clock)
    assert len(done) == 3 and all(n == 1 for _, _, n in eng.calls)


class SleepEngine:
    """A host-only engine whose layers take real time (the concurrent server
    runs one thread per engine on the wall clock)."""

    def __init__(self, layers, cost, work):
        self.layers, self.cost, self.work = layers, cost, work
        self.calls = []

    def n_layers(self, m):
        return self.layers[m]

    def run_layer(self, m, layer, cts):
        import time
        t0 = time.perf_counter()
        time.sleep(self.cost[m])
        self.calls.append((t0, time.perf_counter(), m, layer, len(cts)))
        return [c + [(m, layer)] for c in cts]

    def sync(self):
        pass

    def working_bytes(self, m):
        return self.work[m]


def test_concurrent_server_overlaps_engines_under_one_budget():
    from paper_2409_07751_amd.serve import ConcurrentServer
    engs = [SleepEngine({"a": 3, "b": 2}, {"a": 0.004, "b": 0.006}, {"a": 10, "b": 20}) for _ in range(2)]
    reqs = [Request(i, "ab"[i % 2], [], arrival=0.002 * i, engine=(i // 2) % 2) for i in range(24)]
    srv = ConcurrentServer(engs, hbm_budget=80, max_batch=4)
    peak = []
    orig = srv._admit

    def admit(now):
        orig(now)
        peak.append(srv.in_use)

    srv._admit = admit
    done = srv.run(reqs)
    assert max(peak) <= 80 and max(peak) > 20
    assert len(done) == 24
    for r in done:
        assert r.ct == [(r.model, i) for i in range(engs[r.engine].layers[r.model])]
        assert r.done >= r.arrival
    # each engine ran only its own requests, in batches of at most 4
    for e in engs:
        assert all(n <= 4 for *_, n in e.calls)
    assert sum(n for e in engs for *_, n in e.calls) == sum(e.layers[r.model] for r in done for e in engs[:1])
    # the two engines' layers overlapped in time
    a, b = engs[0].calls, engs[1].calls
    assert any(s0 < e1 and s1 < e0 for s0, e0, *_ in a for s1, e1, *_ in b)
    assert srv.in_use == 0
    rep = latency_report(done, skip=4)
    assert rep["requests"] == 20
