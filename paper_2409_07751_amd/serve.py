"""Continuous-batching server for encrypted KAN inference on one GPU.

Requests (already-encrypted inputs for one of several compiled models) arrive
over time.  The server keeps every admitted request's state on the device
(its current ciphertext and the index of the next layer) and repeatedly runs
one layer for a batch of requests that are at the same layer of the same
model: new arrivals join the next layer-0 batch while earlier requests move
on through later layers, so requests that arrive while others are on the GPU
share launches with them.  Admission is by an HBM budget: a waiting request
enters the active set only if the measured per-request working memory of its
model fits next to the requests already in flight (evaluation keys and
plaintext caches are resident and shared).

The engine interface (`run_layer`, `working_bytes`) is implemented by
`GpuEngine` over the C ABI; tests substitute a host-only engine to check the
scheduler.
"""
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    model: str
    ct: object               # current ciphertext (device handle)
    arrival: float           # seconds from the start of the run
    layer: int = 0
    admitted: float = None
    done: float = None
    batches: list = field(default_factory=list)  # batch sizes this request ran in
    engine: int = 0          # the engine (context) its ciphertext lives in


class GpuEngine:
    """Runs layers through the library; one context, evaluation keys resident."""

    def __init__(self, ctx, keys, models):
        self.ctx, self.keys, self.models = ctx, keys, models  # models: name -> hekan.Model
        self.work = {}

    def n_layers(self, name):
        return self.models[name].n_layers

    def run_layer(self, name, layer, cts):
        return self.ctx.eval_kan_layer_batch(self.models[name], self.keys, layer, cts)

    def sync(self):
        self.ctx.sync()

    def calibrate(self, name, ct):
        """Measure the peak extra device memory of one request through every
        layer of `name` (plaintext caches warm)."""
        self.ctx.sync()
        base = self.ctx.memory(reset_peak=True)["live"]
        x = ct
        for li in range(self.n_layers(name)):
            x = self.run_layer(name, li, [x])[0]
        self.ctx.sync()
        peak = self.ctx.memory()["peak"]
        del x
        self.work[name] = max(peak - base, 1)
        return self.work[name]

    def working_bytes(self, name):
        return self.work[name]


class Server:
    def __init__(self, engine, hbm_budget, max_batch=16):
        self.engine, self.budget, self.max_batch = engine, hbm_budget, max_batch
        self.waiting, self.active, self.finished = [], [], []
        self.in_use = 0
        self.trace = []  # (time, model, layer, batch size)

    def _admit(self, now):
        # FIFO: a request blocked by the budget blocks the ones behind it
        while self.waiting and self.waiting[0].arrival <= now:
            r = self.waiting[0]
            need = self.engine.working_bytes(r.model)
            if self.active and self.in_use + need > self.budget:
                break
            self.waiting.pop(0)
            r.admitted = now
            self.in_use += need
            self.active.append(r)

    def _step(self, now_fn):
        # the (model, layer) group of the oldest active request, batched
        oldest = min(self.active, key=lambda r: (r.arrival, r.rid))
        group = [r for r in self.active if r.model == oldest.model and r.layer == oldest.layer]
        group.sort(key=lambda r: (r.arrival, r.rid))
        batch = group[: self.max_batch]
        outs = self.engine.run_layer(oldest.model, oldest.layer, [r.ct for r in batch])
        self.engine.sync()
        t = now_fn()
        self.trace.append((t, oldest.model, oldest.layer, len(batch)))
        for r, o in zip(batch, outs):
            r.ct = o
            r.layer += 1
            r.batches.append(len(batch))
            if r.layer == self.engine.n_layers(r.model):
                r.done = t
                self.active.remove(r)
                self.in_use -= self.engine.working_bytes(r.model)
                self.finished.append(r)

    def run(self, requests, clock=None):
        """Serve `requests` (arrival times relative to the start); returns the
        finished requests.  `clock` returns seconds since the start (defaults
        to the wall clock)."""
        t0 = time.perf_counter()
        now_fn = clock or (lambda: time.perf_counter() - t0)
        self.waiting = sorted(requests, key=lambda r: (r.arrival, r.rid))
        while self.waiting or self.active:
            now = now_fn()
            self._admit(now)
            if not self.active:
                # idle until the next arrival
                nxt = self.waiting[0].arrival
                if clock is None:
                    time.sleep(max(0.0, nxt - now_fn()))
                else:
                    clock.advance_to(nxt)
                continue
            self._step(now_fn)
        return self.finished


class ConcurrentServer:
    """The same scheduling over several engines, each with its own context,
    HIP stream and resident copy of the evaluation keys, driven by one host
    thread each: a request is bound to the engine its ciphertext was
    encrypted in (`Request.engine`); every thread repeatedly runs the oldest
    (model, layer) group of its own requests as one batch and waits for its
    own stream only, so groups on different engines overlap on the device
    (the library releases the interpreter lock inside every call).
    Admission is shared: one FIFO and one HBM budget for all engines, a
    request entering as soon as memory frees up anywhere."""

    def __init__(self, engines, hbm_budget, max_batch=16):
        self.engines, self.budget, self.max_batch = list(engines), hbm_budget, max_batch
        self.waiting, self.finished = [], []
        self.active = [[] for _ in self.engines]
        self.in_use = 0
        self.trace = []  # (time, engine, model, layer, batch size)
        self.cv = threading.Condition()
        self.error = None

    def _admit(self, now):
        while self.waiting and self.waiting[0].arrival <= now:
            r = self.waiting[0]
            need = self.engines[r.engine].working_bytes(r.model)
            if any(self.active) and self.in_use + need > self.budget:
                break
            self.waiting.pop(0)
            r.admitted = now
            self.in_use += need
            self.active[r.engine].append(r)

    def _worker(self, e, now_fn):
        eng = self.engines[e]
        try:
            while True:
                with self.cv:
                    while True:
                        if self.error is not None:
                            return
                        self._admit(now_fn())
                        if self.active[e]:
                            break
                        if not self.waiting and not any(self.active):
                            self.cv.notify_all()
                            return
                        # sleep until the next arrival, or (nothing left to arrive, or the
                        # head of the queue waiting for memory) until another engine finishes
                        nxt = self.waiting[0].arrival - now_fn() if self.waiting else None
                        self.cv.wait(timeout=None if nxt is None or nxt <= 0 else nxt + 1e-4)
                    act = self.active[e]
                    oldest = min(act, key=lambda r: (r.arrival, r.rid))
                    group = sorted((r for r in act if r.model == oldest.model and r.layer == oldest.layer),
                                   key=lambda r: (r.arrival, r.rid))
                    batch = group[: self.max_batch]
                outs = eng.run_layer(oldest.model, oldest.layer, [r.ct for r in batch])
                eng.sync()
                with self.cv:
                    t = now_fn()
                    self.trace.append((t, e, oldest.model, oldest.layer, len(batch)))
                    for r, o in zip(batch, outs):
                        r.ct = o
                        r.layer += 1
                        r.batches.append(len(batch))
                        if r.layer == eng.n_layers(r.model):
                            r.done = t
                            act.remove(r)
                            self.in_use -= eng.working_bytes(r.model)
                            self.finished.append(r)
                    self.cv.notify_all()
        except BaseException as ex:  # stop every worker, re-raised by run()
            with self.cv:
                self.error = ex
                self.cv.notify_all()

    def run(self, requests):
        t0 = time.perf_counter()
        now_fn = lambda: time.perf_counter() - t0
        self.waiting = sorted(requests, key=lambda r: (r.arrival, r.rid))
        th = [threading.Thread(target=self._worker, args=(e, now_fn)) for e in range(len(self.engines))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if self.error is not None:
            raise self.error
        return self.finished


def hbm_budget(engines, fraction=0.8):
    """An admission budget from the device itself: `fraction` of the memory
    not yet in use once every engine's evaluation keys and plaintext caches
    are resident (the device's free bytes plus the bytes the engines' pools
    hold for reuse)."""
    free = engines[0].ctx.device_memory()["free"]
    cached = sum(e.ctx.memory()["cached"] for e in engines)
    return int(fraction * (free + cached))


def latency_report(finished, skip=0):
    """Per-request latency (arrival to completion) and throughput; `skip`
    leaves out the first requests by arrival (the warm-up before a steady
    state), both from the percentiles and from the throughput window."""
    fin = sorted(finished, key=lambda r: (r.arrival, r.rid))[skip:]
    lat = np.array([r.done - r.arrival for r in fin])
    span = max(r.done for r in fin) - min(r.arrival for r in fin)
    sizes = [b for r in fin for b in r.batches]
    return {"requests": len(fin), "inferences_per_s": round(len(fin) / span, 4),
            "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 2),
            "mean_batch": round(float(np.mean(sizes)), 2), "span_s": round(span, 3)}
