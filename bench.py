"""Encrypted KAN inference benchmark on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B] [--workload image]

A step is one encrypted inference pass of the whole network (SiLU branch,
B-spline bases, fused linear layers, every key switch) over one batch of B
synthetic encrypted inputs that are already resident in HBM.  Prints one
JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Roofline of the timed kernel class: its algorithmic bytes (every word a
# launch must read or write once: inputs, the intermediate between the two
# passes, outputs and the fused policies' extra operands) over its measured
# time, against the 8 TB/s HBM peak.  The default is the largest class of the
# step, the forward column pass (ModUp's and ModDown's basis conversion fused
# into its loads, the rescale input); its limit is instruction issue rather
# than HBM (the conversion's exact FP64 products and the 60-bit primes'
# integer arithmetic), so its HBM fraction is low.  The butterfly rate is
# reported beside it.
HBM_PEAK_GBPS = 8000.0
NTT_KERNELS = ("ntt_fwd_pass1", "ntt_fwd_pass2", "ntt_inv_pass2", "ntt_inv_pass1")
# HBM bytes per launch of the default roofline kernel at the default batch,
# from calibrated FETCH_SIZE + WRITE_SIZE counter runs of this benchmark with
# the default key-switch configuration (--no-autotune: the column pass's
# launches are the same in every configuration, the row pass's are not);
# emptied whenever the kernel changes until the counters are taken again
TRAFFIC_BYTES_PER_LAUNCH = {"ntt_fwd_pass1": 306800000, "ntt_fwd_pass2": 490580000}


def roofline(kernel, prof, batch):
    """Achieved vs peak for the timed kernel from the live HIP-event timings."""
    if prof["launches"] == 0:
        return None
    secs = prof["ms"] * 1e-3
    achieved = prof["bytes"] / secs / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBPS, 4),
         "traffic": TRAFFIC_BYTES_PER_LAUNCH.get(kernel) if batch == 16 else None,
         "algorithmic_bytes_per_launch": round(prof["bytes"] / prof["launches"]),
         "avg_launch_us": round(prof["ms"] * 1e3 / prof["launches"], 3), "launches": prof["launches"]}
    if kernel in NTT_KERNELS:
        r["butterflies_per_s"] = round(prof["ops"] / secs, -6)
    return r


def copy_probe(mib):
    """One device-to-device copy of a known size through the HIP runtime, so a
    counter run can calibrate FETCH_SIZE / WRITE_SIZE."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    n = mib << 20
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(a), ctypes.c_size_t(n)) == 0
    assert hip.hipMalloc(ctypes.byref(b), ctypes.c_size_t(n)) == 0
    assert hip.hipMemset(a, 1, ctypes.c_size_t(n)) == 0
    assert hip.hipMemcpy(b, a, ctypes.c_size_t(n), 3) == 0  # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    log("copy probe: %d MiB device-to-device" % mib)


def cpu_baseline(wl, budget):
    """The CPU oracle (plain C + Python, one thread) on a bounded sample of the
    same workload: it runs the [784,64,10] encrypted inference from its start
    for `budget` seconds (key generation excluded) and the throughput is
    extrapolated from the fraction of the inference's key-switch work done,
    weighting a key switch at level l by its limb-digit count
    ceil((l+1)/w) (l+1+alpha)."""
    from oracle import ckks as O, circuit, kan
    from oracle.slotsim import SlotSim
    from paper_2409_07751_amd import synth

    layers = kan.compile_model(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024),
                               [wl.silu_degree] * (len(wl.shape) - 1), [list(c) for c in wl.comp_degrees],
                               wl.grid, wl.silu_range, prescale=wl.prescale)
    prm = O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)

    def work(l):
        return ((l + 1 + wl.w - 1) // wl.w) * (l + 1 + wl.alpha)

    class Rec(SlotSim):
        def __init__(self, slots):
            super().__init__(slots)
            self.w = 0

        def relin_rescale(self, t):
            self.w += work(t[0])
            return super().relin_rescale(t)

        def rotate(self, a, t):
            if t % self.ctx.p.slots:
                self.w += work(a.level)
            return super().rotate(a, t)

    sim = Rec(prm.slots)
    circuit.eval_kan(sim, sim.fresh(np.zeros(wl.shape[0]), wl.L), layers, circ=circuit.RESTRUCTURED)
    total_work = sim.w

    ctx = O.Context(prm)
    keys = O.Keys.__new__(O.Keys)
    keys.ctx = ctx
    L = O.lib()
    s = np.zeros(prm.N, np.int64)
    L.oc_sample_ternary(3, 1, 0, 0, prm.logN, O.P(s))
    ktot = prm.L + 1 + prm.alpha
    keys.s_res = np.zeros((ktot, prm.N), np.uint64)
    L.oc_small_to_rns(O.P(s), O.P(keys.s_res), ktot, prm.logN, O.P(ctx.all_mods))
    dnum = (prm.L + 1 + prm.w - 1) // prm.w
    state = {"keygen": 0.0, "work": 0, "t0": None}

    class LazyKeys(dict):
        def __missing__(self, g):
            t0 = time.perf_counter()
            sp = np.zeros_like(keys.s_res)
            if g == 0:
                L.oc_poly_mul(O.P(keys.s_res), O.P(keys.s_res), O.P(sp), ktot, prm.logN, O.P(ctx.all_mods))
            else:
                L.oc_automorph(O.P(keys.s_res), O.P(sp), ktot, prm.logN, O.P(ctx.all_mods), g)
            self[g] = keys._gen(3, g, sp, dnum)
            state["keygen"] += time.perf_counter() - t0
            return self[g]

    keys.keys = LazyKeys()

    class Stop(Exception):
        pass

    class Timed(O.Oracle):
        def keyswitch(self, d, l, key_id, galois=0):
            keys.keys[key_id]  # generate outside the measured time
            if time.perf_counter() - state["t0"] - state["keygen"] > budget:
                raise Stop()
            r = super().keyswitch(d, l, key_id, galois)
            state["work"] += work(l)
            return r

    ev = Timed(ctx, keys)
    x = synth.inputs(wl, 1)[0]
    ct = ev.encrypt(x, synth.SEED_ENC)
    log("cpu baseline: oracle running the inference for %.0f s" % budget)
    state["t0"] = time.perf_counter()
    try:
        circuit.eval_kan(ev, ct, layers, circ=circuit.RESTRUCTURED)
    except Stop:
        pass
    elapsed = time.perf_counter() - state["t0"] - state["keygen"]
    frac = state["work"] / total_work
    log("cpu baseline: %.4f of the key-switch work in %.1f s" % (frac, elapsed))
    return {"value": round(frac / elapsed, 6), "unit": "inferences/s", "cores": 1, "kind": "oracle",
            "sample": "first %.0f s of one [784,64,10] inference on the single-threaded CPU oracle "
                      "(%d key switches, %.2f%% of the inference's key-switch work, key generation excluded); "
                      "extrapolated by key-switch work" % (elapsed, ev.count["ks"], 100 * frac)}


def plain_path(ctx, model, keys, ct, steps):
    """The per-ciphertext path: one inference at a time, same kernels."""
    ctx.eval_kan(model, keys, ct)
    ctx.sync()
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        out = ctx.eval_kan(model, keys, ct)
        ctx.sync()
        lat.append(time.perf_counter() - t0)
        del out
    lat = np.array(lat)
    return {"inferences_per_s": round(steps / lat.sum(), 4), "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3), "steps": steps}


def graph_path(ctx, model, keys, cts, steps, want, n_out):
    """The same inference captured once into a HIP graph and replayed (the
    host's launch cost off the device's critical path): inferences/s over
    `steps` replays for this batch, and the replayed result's accuracy."""
    graph, outs = ctx.capture_kan_batch(model, keys, cts)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    ctx.sync()
    elapsed = time.perf_counter() - t0
    err = max(float(np.abs(ctx.decrypt(keys, outs[i], n_out) - want[i]).max()) for i in range(len(cts)))
    graph.free()
    del outs
    return {"batch": len(cts), "inferences_per_s": round(len(cts) * steps / elapsed, 4),
            "ms_per_replay": round(elapsed / steps * 1e3, 3), "replays": steps, "max_abs_err_vs_fp64_circuit": err}


SERVE_MIX = (("formula16", 0.5), ("image", 0.3), ("cifar", 0.2))


def serve_run(args, batched_rate):
    """Requests drawn from the serving mix on one context with every model's
    keys resident: (1) Poisson arrivals at 0.7x the measured batched image
    throughput, served with layer-granular continuous batching under an HBM
    budget (p50/p99 latency, inferences/s); (2) the mixed batch: 64 requests
    present at once under a 96 GiB budget, grouped by (model, layer) into
    launches of up to 32."""
    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth
    from paper_2409_07751_amd.serve import GpuEngine, Request, Server, latency_report

    names = [n for n, _ in SERVE_MIX]
    probs = np.array([p for _, p in SERVE_MIX])
    wl0 = synth.WORKLOADS["image"]
    ctx = hekan.Context(wl0.logN, wl0.L, wl0.scale_bits, wl0.alpha, wl0.w)
    layers, models = {}, {}
    for n in names:
        wl = synth.WORKLOADS[n]
        layers[n] = pc.compile_kan(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024), wl.silu_degree,
                                   [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
        models[n] = ctx.compile(layers[n])
    steps = sorted(set(s for m in models.values() for s in m.rotation_steps()))
    t0 = time.time()
    keys = ctx.keygen(synth.SEED_KEYGEN, steps)
    ctx.sync()
    log("serving keygen %.1fs (%d Galois keys)" % (time.time() - t0, len(steps)))
    eng = GpuEngine(ctx, keys, models)
    for n in names:
        x = synth.inputs(synth.WORKLOADS[n], 1, stream=3)[0]
        eng.calibrate(n, ctx.encrypt_input(models[n], keys, x, 7))
    free = ctx.memory()
    budget = 40 * 2 ** 30

    def make(nreq, arrivals, stream0):
        kinds = synth.request_mix(nreq, names, probs, seed=synth.SEED_ARRIVALS + stream0)
        reqs = []
        for i, n in enumerate(kinds):
            x = synth.inputs(synth.WORKLOADS[n], 1, stream=stream0 + i)[0]
            reqs.append(Request(i, n, ctx.encrypt_input(models[n], keys, x, 1000 + 10 * i), float(arrivals[i])))
        ctx.sync()
        return reqs

    rate = 0.7 * batched_rate
    nreq = args.serve_requests
    reqs = make(nreq, synth.poisson_arrivals(rate, nreq), 100)
    log("serving %d requests at %.1f/s, budget %.1f GiB (pool live %.1f GiB)" % (nreq, rate, budget / 2 ** 30,
                                                                                 free["live"] / 2 ** 30))
    done = Server(eng, budget, max_batch=args.serve_batch).run(reqs)
    rep = latency_report(done)
    rep.update({"arrival_rate_per_s": round(rate, 3), "mix": {n: float(p) for n, p in zip(names, probs)},
                "hbm_budget_GiB": budget / 2 ** 30,
                "working_MiB_per_request": {n: round(eng.work[n] / 2 ** 20, 1) for n in names}})
    log("serving:", rep)
    del reqs, done

    reqs = make(64, np.zeros(64), 5000)
    log("mixed batch of 64 requests")
    t0 = time.perf_counter()
    done = Server(eng, 96 * 2 ** 30, max_batch=32).run(reqs)
    ctx.sync()
    span = time.perf_counter() - t0
    kinds = {n: sum(1 for r in done if r.model == n) for n in names}
    mixed = {"requests": len(done), "inferences_per_s": round(len(done) / span, 3), "span_s": round(span, 3),
             "mean_batch": latency_report(done)["mean_batch"], "per_model": kinds}
    log("mixed batch:", mixed)
    del reqs, done, keys, models, eng
    ctx.close()
    return rep, mixed


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="steps of the plain per-ciphertext path (batch 1) timed for comparison; 0 skips")
    ap.add_argument("--workload", default="image")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="replays of the inference captured into a HIP graph, at the batch and at batch 1 (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--roofline-kernel", default="ntt_fwd_pass1")
    ap.add_argument("--no-serve", action="store_true", help="skip the continuous-batching server run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default key-switch configuration (fused, spans of 8) at every level")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): requests are independent, so N GPUs would "
              "serve N queues, each with its own copy of the evaluation keys and no exchange on the "
              "hot path", file=sys.stderr)
        sys.exit(2)

    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth

    wl = synth.WORKLOADS[args.workload]
    log("workload", wl.name, "N=2^%d" % wl.logN, "L=%d" % wl.L, "shape", wl.shape)
    raw = synth.raw_weights(wl)
    layers = pc.compile_kan(raw, synth.calibration_inputs(wl, 1024), wl.silu_degree,
                            [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    ctx = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    model = ctx.compile(layers)
    steps = model.rotation_steps()
    t0 = time.time()
    keys = ctx.keygen(synth.SEED_KEYGEN, steps)
    ctx.sync()
    log("keygen %.1fs (%d Galois keys)" % (time.time() - t0, len(steps)))
    B = args.batch
    x = synth.inputs(wl, B)
    cts = [ctx.encrypt(keys, x[i], synth.SEED_ENC + i) for i in range(B)]
    ctx.sync()

    def step():
        outs = ctx.eval_kan_batch(model, keys, cts)
        ctx.sync()
        return outs

    # key-switch configuration per level, chosen by measurement for the timed
    # batch and for the plain path's batch of one
    tune = {}
    if not args.no_autotune:
        t0 = time.time()
        for nb in sorted({B, 1}):
            tune[str(nb)] = ctx.autotune(keys, nb)
        log("key-switch autotune %.1fs: %s" % (time.time() - t0, tune))

    for w in range(args.warmup):
        t0 = time.time()
        outs = step()
        log("warmup %d: %.3fs" % (w, time.time() - t0))
    # accuracy check of the last warmup output against the plain FP64 circuit
    want = pc.plain_forward(x, layers)
    err = max(float(np.abs(ctx.decrypt(keys, outs[i], wl.shape[-1]) - want[i]).max()) for i in range(B))
    log("max |decrypt - fp64 circuit| = %.3e" % err)
    del outs

    c0 = ctx.counters()
    lat = []
    ctx.sync()
    ctx.profile(args.roofline_kernel)
    t_start = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        outs = step()
        lat.append(time.perf_counter() - t0)
        del outs
    ctx.sync()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile_read()
    ctx.profile(None)
    c1 = ctx.counters()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    roof = roofline(args.roofline_kernel, prof, B)
    ks_per_step = (c1["keyswitches"] - c0["keyswitches"]) / args.steps
    inf_s = B * args.steps / elapsed
    lat_ms = np.array(lat) * 1e3
    res = {
        "metric": "encrypted KAN inferences/s (N=2^16)",
        "value": round(inf_s, 4),
        "unit": "inferences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "KAN [784,64,10] encrypted inference, RNS-CKKS N=2^16, L=24, 4 special primes, "
                               "5-limb digits", "batch": B, "levels": wl.L, "log_n": wl.logN},
        "keyswitches_per_s": round(ks_per_step * args.steps / elapsed, 1),
        "keyswitches_per_inference": ks_per_step / B,
        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "max_abs_err_vs_fp64_circuit": err,
        "launches_per_step": (c1["launches"] - c0["launches"]) / args.steps,
        "roofline": roof,
        "keyswitch_autotune": tune or None,
    }
    if args.plain_steps:
        res["plain_path"] = plain_path(ctx, model, keys, cts[0], args.plain_steps)
        res["batched_vs_plain"] = round(res["value"] / res["plain_path"]["inferences_per_s"], 3)
    if args.graph_steps:
        res["graph_path"] = [graph_path(ctx, model, keys, c, args.graph_steps, want, wl.shape[-1])
                             for c in (cts, cts[:1])]
    if not args.no_serve:
        res["serving"], res["batched_mix"] = serve_run(args, res["value"])
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    del cts, keys, model
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
