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
TRAFFIC_BYTES_PER_LAUNCH = {"ntt_fwd_pass1": 308730000, "ntt_fwd_pass2": 482820000}
TRAFFIC_SOURCE = "profiles/%s_image_b16_hbm_traffic.md (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated by a copy)"
# Instruction issue of the same launches: wave64 VALU instructions per launch
# (rocprofv3 SQ_INSTS_VALU summed over the class's dispatches of one timed
# step, over their number) against the issue peak: each of a CU's 4 SIMDs
# starts one wave64 VALU instruction every 4 cycles (16 lanes a cycle; the
# FP64 FMA peak of 78.6 TFLOP/s = 2 x 64 lanes x this rate), i.e.
# 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G instructions/s.  Emptied whenever
# the kernel changes until the counters are taken again.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
VALU_INSTS_PER_LAUNCH = {"ntt_fwd_pass1": 62606796, "ntt_fwd_pass2": 36462952}
VALU_SOURCE = "profiles/%s_image_b16_valu.md (rocprofv3 SQ_INSTS_VALU)"


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
    if r["traffic"] is not None:
        r["traffic_source"] = TRAFFIC_SOURCE % kernel
    if kernel in NTT_KERNELS:
        r["butterflies_per_s"] = round(prof["ops"] / secs, -6)
    insts = VALU_INSTS_PER_LAUNCH.get(kernel) if batch == 16 else None
    if insts:
        rate = insts / (secs / prof["launches"])
        r["compute"] = {"bound": "valu_issue", "insts_per_launch": insts, "achieved": round(rate / 1e9, 1),
                        "peak": VALU_ISSUE_PEAK / 1e9, "unit": "G wave64 VALU instructions/s",
                        "frac": round(rate / VALU_ISSUE_PEAK, 4), "source": VALU_SOURCE % kernel}
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


def cpu_baseline(wl):
    """The CPU oracle as it stands (plain C + Python, OpenMP over RNS limbs) on
    the host cores: one whole encrypted [784,64,10] inference of the
    benchmark's circuit on one input (key generation timed apart, outside the
    inference), with every host thread the oracle uses; the [2,5,1] (one
    input) and [4,10,10,1] (64 vectors in one ciphertext) inferences at their
    own parameters with the client-aided refresh, likewise; then, on one thread
    (the paper's single-thread setting), one forward limb NTT at N = 2^13,
    2^15 and 2^16 and one relinearised product and one rotation at the top
    level."""
    from oracle import ckks as O, circuit, kan
    from paper_2409_07751_amd import synth

    layers = kan.compile_model(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024),
                               [wl.silu_degree] * (len(wl.shape) - 1), [list(c) for c in wl.comp_degrees],
                               wl.grid, wl.silu_range, prescale=wl.prescale)
    prm = O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    ctx = O.Context(prm)
    O.set_threads(0)
    threads = O.get_threads()
    steps = circuit.rotation_steps(layers, prm.slots, circ=circuit.RESTRUCTURED)
    t0 = time.perf_counter()
    ev = O.Oracle(ctx, O.Keys(ctx, synth.SEED_KEYGEN, steps))
    keygen_s = time.perf_counter() - t0
    x = synth.inputs(wl, 1)[0]
    ct = ev.encrypt(x, synth.SEED_ENC)
    log("cpu baseline: oracle inference on %d threads (keygen %.1f s)" % (threads, keygen_s))
    t0 = time.perf_counter()
    out = circuit.eval_kan(ev, ct, layers, circ=circuit.RESTRUCTURED)
    inf_s = time.perf_counter() - t0
    n_ks = ev.count["ks"]
    y = ev.decrypt(out, wl.shape[-1])
    err = float(np.abs(y - kan.he_friendly_kan(x[None], layers)[0]).max())
    log("cpu baseline: one inference in %.1f s (%d key switches), max err %.2e" % (inf_s, n_ks, err))
    # the two smaller configurations run fully (client-aided refresh between
    # layers, as on the GPU at their parameters), all threads
    full = {}
    for name, S in (("tiny", 1), ("formula", 64)):
        w2 = synth.WORKLOADS[name]
        lay = kan.compile_model(synth.raw_weights(w2), synth.calibration_inputs(w2, 1024),
                                [w2.silu_degree] * (len(w2.shape) - 1), [list(c) for c in w2.comp_degrees],
                                w2.grid, w2.silu_range, prescale=w2.prescale)
        c2 = O.Context(O.Params(w2.logN, w2.L, w2.scale_bits, w2.alpha, w2.w))
        e2 = O.Oracle(c2, O.Keys(c2, synth.SEED_KEYGEN,
                                 circuit.rotation_steps(lay, c2.p.slots, S, circ=circuit.RESTRUCTURED)))
        X = synth.inputs(w2, S)
        c_in = e2.encrypt(circuit.pack_samples(X, S) if S > 1 else X[0], synth.SEED_ENC)
        t0 = time.perf_counter()
        o2 = circuit.eval_kan(e2, c_in, lay, S=S, circ=circuit.RESTRUCTURED,
                              refresh=lambda c, li: e2.encrypt(e2.decrypt(c, c2.p.slots), 300 + li))
        full[name] = {"s": round(time.perf_counter() - t0, 2), "vectors": S, "key_switches": e2.count["ks"],
                      "n": 1 << w2.logN}
        del e2, c2, o2
    log("cpu baseline, configurations 0-1 in full:", full)
    # one thread
    O.set_threads(1)
    L = O.lib()
    ntt = {}
    for logn in (13, 15, 16):
        q = int(O.Context(O.Params(logn, 1, 40, 1, 1)).q[1])
        a = np.random.default_rng(logn).integers(0, q, 1 << logn, dtype=np.uint64)
        t0 = time.perf_counter()
        for _ in range(5):
            L.oc_ntt_fwd(O.P(a), logn, q)
        ntt["2^%d" % logn] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
    rng = np.random.default_rng(7)
    A = [np.array([rng.integers(0, int(ctx.q[l]), prm.N, dtype=np.uint64) for l in range(prm.L + 1)])
         for _ in range(4)]
    ca, cb = O.Ciphertext(prm.L, A[0], A[1]), O.Ciphertext(prm.L, A[2], A[3])
    t0 = time.perf_counter()
    ev.mul(ca, cb)
    mul_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ev.rotate(ca, steps[-1] if steps[-1] > 0 else 1)
    rot_s = time.perf_counter() - t0
    O.set_threads(0)
    log("cpu baseline, one thread: top-level product %.2f s, rotation %.2f s" % (mul_s, rot_s))
    return {"value": round(1.0 / inf_s, 6), "unit": "inferences/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(),
            "sample": "one whole [784,64,10] encrypted inference (batch 1, the benchmark's circuit: %d key switches) "
                      "on the CPU oracle with %d OpenMP threads over RNS limbs; key generation (%.1f s) "
                      "excluded; decrypted within %.1e of the FP64 circuit" % (n_ks, threads, keygen_s, err),
            "inference_s": round(inf_s, 2), "keygen_s": round(keygen_s, 2),
            "single_thread": {"ntt_ms": ntt, "relinearised_product_top_level_s": round(mul_s, 3),
                              "rotation_top_level_s": round(rot_s, 3)},
            "configs_0_1_full_inference": full}


# chains of the same ring with every prime below 2^46, so every limb runs on
# exact FP64 words: 46-bit q_0, 5 special primes of 46 bits and 5-limb digits
# (the largest digit, 46 + 4 x 45 bits, stays below P's 230 bits).  The
# logits (up to about 3) exceed what level 0 holds with a 46-bit q_0
# (q_0 / (2 S) = 1), so either one more 45-bit level keeps the output at
# level 1 (26 + 5 limbs and 6 digits at the top, against the workload's 25 + 4
# and 5), or the last layer's weights are scaled by 1/4 and the decrypted
# logits by 4 (the same 24 levels: 25 + 5 limbs, 5 digits)
ALL_FP64_CHAINS = ((1, 1.0), (0, 4.0))  # (extra levels, output scale)


def word_study(args, layers, wl, x, want):
    """The batched inference (one engine, batch 16) with the default words
    (primes below 2^46 in exact FP64 arithmetic, the 60-bit primes on 64-bit
    integer words), with every prime on 64-bit integer words (Shoup
    butterflies, Barrett and Montgomery products; the FP64 path off), and on
    chains whose primes are all below 2^46 (ALL_FP64_CHAINS: every limb on
    FP64, at the price of more limbs): inferences/s of each.  The first two
    compute the same residues."""
    import dataclasses
    from paper_2409_07751_amd import hekan, synth
    out = {"batch": 16, "all_primes_below_2^46": []}
    variants = [("fp64_path", (wl.L, wl.alpha, wl.w), {}, 1.0),
                ("integer_words", (wl.L, wl.alpha, wl.w), {"integer_words": True}, 1.0)]
    variants += [("all_primes_below_2^46", (wl.L + extra, 5, 5), {"base_bits": 46, "special_bits": 46}, osc)
                 for extra, osc in ALL_FP64_CHAINS]
    for name, (L, alpha, dw), kw, osc in variants:
        ctx = hekan.Context(wl.logN, L, wl.scale_bits, alpha, dw, **kw)
        ls = layers
        if osc != 1.0:
            ls = list(layers[:-1]) + [dataclasses.replace(layers[-1], wb=layers[-1].wb / osc, ws=layers[-1].ws / osc)]
        model = ctx.compile(ls)
        keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
        cts = [ctx.encrypt(keys, x[i], synth.SEED_ENC + i) for i in range(16)]
        outs = ctx.eval_kan_batch(model, keys, cts)
        ctx.sync()
        err = max(float(np.abs(osc * ctx.decrypt(keys, outs[i], wl.shape[-1]) - want[i]).max()) for i in range(16))
        out_level = outs[0].level
        del outs
        steps = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps):
            outs = ctx.eval_kan_batch(model, keys, cts)
            del outs
        ctx.sync()
        el = time.perf_counter() - t0
        r = {"inferences_per_s": round(16 * steps / el, 4), "steps": steps, "max_abs_err_vs_fp64_circuit": err}
        if kw.get("base_bits"):
            q, pm, _ = ctx.primes()
            r["chain"] = "%d-bit q_0 + %d x %d-bit, %d x %d-bit special primes, %d-limb digits" % (
                int(q[0]).bit_length(), L, wl.scale_bits, alpha, int(pm[0]).bit_length(), dw)
            r["output_level"] = out_level
            if osc != 1.0:
                r["output_scale"] = "last layer's weights / %g, decrypted logits x %g" % (osc, osc)
            out[name].append(r)
        else:
            out[name] = r
        del cts, keys, model
        ctx.close()
    return out


def silu_fits():
    """The SiLU approximation comparators (host side): the weighted
    least-squares fit, ordinary least squares and Remez minimax at one degree
    and range, measured by the RMSE over the range and over a synthetic
    activation distribution.  Ranges and degrees are the ones the paper's
    experiments state for its three image data sets (5-sigma ranges; degrees
    10, 10, 15), with normal activations of that mean and sigma; plus the
    hidden-layer activations of the [784,64,10] model (calibration inputs
    through its first layer) at its degree 31."""
    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import synth
    out = {}
    for name, (lo, hi, deg) in (("range_mnist", (-12.4, 14.74, 10)), ("range_fmnist", (-9.77, 11.01, 10)),
                                ("range_cifar10", (-11.90, 10.99, 15))):
        mu, sd = (lo + hi) / 2, (hi - lo) / 10
        samples = np.random.default_rng(synth.SEED_CALIB).normal(mu, sd, 200000)
        out[name] = {"lo": lo, "hi": hi, "degree": deg, "fits": pc.silu_fit_comparison(lo, hi, deg, samples)}
    wl = synth.WORKLOADS["image"]
    raw = synth.raw_weights(wl)
    calib = synth.calibration_inputs(wl, 1024)
    layers = pc.compile_kan(raw, calib, wl.silu_degree, [list(c) for c in wl.comp_degrees], wl.grid,
                            wl.silu_range, prescale=wl.prescale)
    h = pc.plain_layer(calib, layers[0]).ravel()
    L1 = layers[1]
    out["image_hidden_layer"] = {"lo": L1.silu_lo, "hi": L1.silu_hi, "degree": wl.silu_degree,
                                 "fits": pc.silu_fit_comparison(L1.silu_lo, L1.silu_hi, wl.silu_degree, h)}
    for v in out.values():
        for f in v["fits"].values():
            for k in f:
                f[k] = float("%.5g" % f[k])
    return out


def ks_bench(ctx, keys, wl, keys_steps):
    """Key switches of B = 1, 8 and 64 ciphertexts sharing one key, at every
    level: the relinearisation of a product (with its rescale, as the library
    runs it) and a rotation by one slot; key switches per second and the
    median time of one batch (HIP events on the library stream)."""
    out = {"unit": "keyswitches/s", "levels": list(range(wl.L, -1, -1)), "reps": 5}
    for B in (1, 8, 64):
        row = {}
        for kind, st in (("relinearisation", 0), ("rotation", 1)):
            rate = []
            for lvl in out["levels"]:
                if st == 0 and lvl == 0:
                    rate.append(None)
                    continue
                ms = ctx.bench_keyswitch(keys, st, lvl, B, 5)
                rate.append(round(B / (ms * 1e-3), 1))
            row[kind] = rate
        row["top_level_us_per_keyswitch"] = {k: round(1e6 / v[0], 2) for k, v in row.items()}
        out["batch_%d" % B] = row
        log("keyswitch bench B=%d top level: %s keyswitches/s" % (B, {k: v[0] for k, v in row.items()
                                                                      if isinstance(v, list)}))
    # B = 8 distinct keys: one top-level ciphertext rotated by 8 different steps,
    # one key switch (one launch sequence) per key
    from paper_2409_07751_amd import synth
    steps = [s for s in keys_steps if s > 0][:8]
    ct = ctx.encrypt(keys, np.zeros(4), synth.SEED_ENC)
    for s in steps:
        ctx.rotate(keys, ct, s)
    ctx.sync()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        outs = [ctx.rotate(keys, ct, s) for s in steps]
        del outs
    ctx.sync()
    el = time.perf_counter() - t0
    out["distinct_keys_8_top_level"] = {"rotation_keyswitches_per_s": round(reps * len(steps) / el, 1),
                                        "steps": steps, "note": "one ciphertext, 8 keys, one key switch each"}
    return out


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
# the batched configuration's own mix: uniform over three uneven shapes
MIX64 = (("tiny16", 1 / 3), ("formula16", 1 / 3), ("cifar", 1 / 3))


def serve_run(args):
    """Serving on engines (contexts with their own HIP stream and resident
    copy of every model's evaluation keys) driven by one host thread each,
    requests bound to engines round-robin:
      (1) the serving mix 50/30/20 of [4,10,10,1] / [784,64,10] /
          [3072,128,10], all requests present at once: its saturation
          throughput;
      (2) Poisson arrivals of the same mix at 0.7 x that throughput, served
          with layer-granular continuous batching under an HBM budget:
          per-request p50/p99 latency and inferences/s in steady state (the
          first 10% of the requests by arrival left out);
      (3) the batched configuration's mix: 64 requests drawn uniformly from
          [2,5,1] / [4,10,10,1] / [3072,128,10] (seed 5), all present at
          once, in launches of up to 32 per (model, layer) group."""
    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth
    from paper_2409_07751_amd.serve import ConcurrentServer, GpuEngine, Request, hbm_budget, latency_report

    names = sorted(set(n for n, _ in SERVE_MIX + MIX64))
    wl0 = synth.WORKLOADS["image"]
    layers = {}
    for n in names:
        wl = synth.WORKLOADS[n]
        layers[n] = pc.compile_kan(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024), wl.silu_degree,
                                   [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    engines = []
    for e in range(args.serve_engines):
        ctx = hekan.Context(wl0.logN, wl0.L, wl0.scale_bits, wl0.alpha, wl0.w)
        models = {n: ctx.compile(layers[n]) for n in names}
        steps = sorted(set(s for m in models.values() for s in m.rotation_steps()))
        t0 = time.time()
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        ctx.sync()
        log("serving engine %d: keygen %.1fs (%d Galois keys)" % (e, time.time() - t0, len(steps)))
        eng = GpuEngine(ctx, keys, models)
        for n in names:
            x = synth.inputs(synth.WORKLOADS[n], 1, stream=3)[0]
            eng.calibrate(n, ctx.encrypt_input(models[n], keys, x, 7))
        engines.append(eng)

    def make(nreq, arrivals, mix, stream0):
        kinds = synth.request_mix(nreq, [n for n, _ in mix], np.array([p for _, p in mix]),
                                  seed=synth.SEED_ARRIVALS + stream0)
        reqs = []
        for i, n in enumerate(kinds):
            eng = engines[i % len(engines)]
            x = synth.inputs(synth.WORKLOADS[n], 1, stream=stream0 + i)[0]
            ct = eng.ctx.encrypt_input(eng.models[n], eng.keys, x, 1000 + 10 * i)
            reqs.append(Request(i, n, ct, float(arrivals[i]), engine=i % len(engines)))
        for eng in engines:
            eng.ctx.sync()
        return reqs

    def saturated(nreq, mix, stream0, max_batch):
        reqs = make(nreq, np.zeros(nreq), mix, stream0)
        t0 = time.perf_counter()
        done = ConcurrentServer(engines, hbm_budget(engines), max_batch=max_batch).run(reqs)
        span = time.perf_counter() - t0
        out = {"requests": len(done), "inferences_per_s": round(len(done) / span, 3), "span_s": round(span, 3),
               "mean_batch": latency_report(done)["mean_batch"],
               "per_model": {n: sum(1 for r in done if r.model == n) for n, _ in mix},
               "engines": len(engines)}
        del reqs, done
        return out

    # each measurement follows a warm-up pass of the same requests (the
    # engines' buffer pools and plaintext caches as in steady state)
    log("serving mix, saturation: %d requests at once" % args.serve_saturation)
    saturated(args.serve_saturation, SERVE_MIX, 3000, args.serve_batch)
    sat = saturated(args.serve_saturation, SERVE_MIX, 3000, args.serve_batch)
    log("serving mix saturation:", sat)
    rate = 0.7 * sat["inferences_per_s"]
    nreq = args.serve_requests
    budget = hbm_budget(engines)
    reqs = make(nreq, synth.poisson_arrivals(rate, nreq), SERVE_MIX, 100)
    log("serving %d requests at %.1f/s, budget %.1f GiB" % (nreq, rate, budget / 2 ** 30))
    done = ConcurrentServer(engines, budget, max_batch=args.serve_batch).run(reqs)
    rep = latency_report(done, skip=nreq // 10)
    rep.update({"arrival_rate_per_s": round(rate, 3), "saturation_inferences_per_s": sat["inferences_per_s"],
                "mix": {n: float(p) for n, p in SERVE_MIX}, "hbm_budget_GiB": round(budget / 2 ** 30, 1),
                "hbm_budget": "0.8 of the device memory free with every engine's keys resident",
                "engines": len(engines), "warmup_requests_excluded": nreq // 10,
                "latency": "per request, arrival to completion",
                "working_MiB_per_request": {n: round(engines[0].work[n] / 2 ** 20, 1) for n, _ in SERVE_MIX}})
    log("serving:", rep)
    del reqs, done

    # the library's native server (he_submit / he_poll) on engine 0: the same
    # mix at once, then Poisson arrivals at 0.7 of its saturation
    eng = engines[0]
    ctx0 = eng.ctx

    def native(nreq, arrivals, stream0):
        kinds = synth.request_mix(nreq, [n for n, _ in SERVE_MIX], np.array([p for _, p in SERVE_MIX]),
                                  seed=synth.SEED_ARRIVALS + stream0)
        cts = [ctx0.encrypt_input(eng.models[n], eng.keys, synth.inputs(synth.WORKLOADS[n], 1, stream=stream0 + i)[0],
                                  1000 + 10 * i) for i, n in enumerate(kinds)]
        ctx0.sync()
        srv = hekan.NativeServer(ctx0, eng.keys, max_batch=args.serve_batch, hbm_budget=hbm_budget(engines[:1]))
        t0 = time.perf_counter()
        tags = []
        for i, n in enumerate(kinds):
            dt = arrivals[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tags.append(srv.submit(eng.models[n], cts[i]))
        lat = [srv.poll(t, wait_ms=600000)[1] for t in tags]
        span = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        skip = nreq // 10 if arrivals[-1] > 0 else 0
        lat = np.array(lat[skip:])
        return {"requests": nreq, "inferences_per_s": round(nreq / span, 3), "span_s": round(span, 3),
                "latency_ms_p50": round(float(np.percentile(lat, 50)), 2),
                "latency_ms_p99": round(float(np.percentile(lat, 99)), 2),
                "mean_batch": round(st["layer_runs"] / max(1, st["layer_batches"]), 2)}

    native(args.serve_saturation, np.zeros(args.serve_saturation), 3000)
    nsat = native(args.serve_saturation, np.zeros(args.serve_saturation), 3000)
    nrate = 0.7 * nsat["inferences_per_s"]
    nserve = native(args.native_requests, synth.poisson_arrivals(nrate, args.native_requests, seed=synth.SEED_ARRIVALS + 7),
                    7000)
    nserve.update({"arrival_rate_per_s": round(nrate, 3), "saturation_inferences_per_s": nsat["inferences_per_s"],
                   "engines": 1, "latency": "per request, submission to completion (measured by the library)",
                   "warmup_requests_excluded": args.native_requests // 10})
    rep["native_server"] = nserve
    log("native server:", nserve)

    log("batched mix of 64 requests of uneven shapes")
    saturated(64, MIX64, 5000, 32)
    mixed = saturated(64, MIX64, 5000, 32)
    log("batched mix:", mixed)
    for eng in engines:
        ctx = eng.ctx
        del eng.keys, eng.models
        ctx.close()
    return rep, mixed


TABLE3_SHAPES = ((64, 3, 2), (128, 5, 3), (256, 5, 3), (256, 10, 3), (256, 10, 5))


# slot counts of the sparsely packed refreshes the bootstrapping block times,
# and of the sparse real-slot one (also the formula KAN's, whose layer outputs
# repeat with period 16)
BOOT_SPARSE_SLOTS = (512, 4096)
BOOT_SPARSE_REAL_SLOTS = 64


def boot_bench(args):
    """CKKS bootstrapping at N = 2^16 (the boot16 parameter set): ms per refresh
    of one ciphertext and refreshes/s in batches, its key switches and levels,
    the decrypted error, and the [4,10,10,1] formula KAN with a bootstrapping
    between layers (the whole inference on the server) against the FP64
    circuit."""
    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth
    bs = synth.BOOTSETS["boot16"]
    ctx = hekan.Context(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, base_bits=bs.base_bits,
                        special_bits=bs.special_bits, sigma=bs.sigma, boot_levels=bs.boot_levels,
                        boot_bits=bs.boot_bits, hamming_weight=bs.h)
    plan = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, pc.boot_cos_coeffs(bs.K, bs.r, bs.degree))
    wl = synth.WORKLOADS["formula16"]
    raw = synth.raw_weights(wl)
    layers = pc.compile_kan(raw, synth.calibration_inputs(wl, 1024), wl.silu_degree,
                            [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    model = ctx.compile(layers, refresh=True, circuit=hekan.CIRCUIT_RESTRUCTURED)
    # the real-slot refresh (SlotToCoeff first)
    rplan = ctx.boot(bs.cts, bs.real_stc, bs.K, bs.r, pc.boot_cos_coeffs(bs.K, bs.r, bs.degree), real_slots=True)
    # sparsely packed refreshes of n-periodic slot vectors
    splans = {n: ctx.boot(bs.cts, bs.stc, bs.K, bs.r, pc.boot_cos_coeffs(bs.K, bs.r, bs.degree), slots=n)
              for n in BOOT_SPARSE_SLOTS}
    # and of real n-periodic slot vectors, SlotToCoeff first
    n_real = BOOT_SPARSE_REAL_SLOTS
    srplan = ctx.boot(bs.cts, bs.real_stc, bs.K, bs.r, pc.boot_cos_coeffs(bs.K, bs.r, bs.degree), real_slots=True,
                      slots=n_real)
    t0 = time.time()
    keys = ctx.keygen(synth.SEED_KEYGEN, sorted(set(plan.rotation_steps()) | set(rplan.rotation_steps()) |
                                                set(model.rotation_steps()) |
                                                set(s for sp in splans.values() for s in sp.rotation_steps()) |
                                                set(srplan.rotation_steps())))
    ctx.sync()
    log("bootstrapping: keygen %.1fs" % (time.time() - t0))
    B = args.boot_batch
    z = synth.boot_inputs(bs, B)
    cts = [ctx.encrypt(keys, z[i], synth.SEED_ENC + i) for i in range(B)]
    t0 = time.time()
    out = ctx.bootstrap(plan, keys, cts[0])
    ctx.sync()
    first = time.time() - t0
    if args.boot_profile:
        # refreshes of one ciphertext separated by idle gaps (for a kernel trace)
        pp, c_in = plan, cts[0]
        if args.boot_profile_plan == "sparse_real":
            n = BOOT_SPARSE_REAL_SLOTS
            pp = srplan
            c_in = ctx.mod_drop(ctx.encrypt(keys, np.tile(z[0][:n], (1 << (bs.logN - 1)) // n), 300), bs.real_stc)
            out = ctx.bootstrap(pp, keys, c_in)
            ctx.sync()
        del rplan
        l0 = ctx.counters()["launches"]
        for _ in range(args.boot_reps):
            time.sleep(0.2)
            out = ctx.bootstrap(pp, keys, c_in)
            ctx.sync()
        log("bootstrapping profile: %d refreshes, %.0f launches each" %
            (args.boot_reps, (ctx.counters()["launches"] - l0) / args.boot_reps))
        del out, cts, keys, model, plan
        ctx.close()
        return {"profile_refreshes": args.boot_reps}
    err = float(np.abs(ctx.decrypt(keys, out, z.shape[1]) - z[0]).max())
    k0 = ctx.counters()["keyswitches"]
    ctx.sync()
    t0 = time.time()
    for _ in range(args.boot_reps):
        out = ctx.bootstrap(plan, keys, cts[0])
    ctx.sync()
    single = (time.time() - t0) / args.boot_reps
    ks = (ctx.counters()["keyswitches"] - k0) / args.boot_reps
    # the stages on their own (CoeffToSlot of the input; EvalMod and SlotToCoeff
    # of ciphertexts at the levels they take in a refresh)
    stages = {}
    w = ctx.boot_coeff_to_slot(plan, keys, cts[0])
    y = ctx.boot_eval_mod(plan, keys, w)
    r = None
    for name, fn in (("coeff_to_slot", lambda: ctx.boot_coeff_to_slot(plan, keys, cts[0])),
                     ("eval_mod_one_half", lambda: ctx.boot_eval_mod(plan, keys, w)),
                     ("slot_to_coeff", lambda: ctx.boot_slot_to_coeff(plan, keys, y, cts[0].level))):
        ctx.sync()
        t0 = time.time()
        for _ in range(args.boot_reps):
            r = fn()
        ctx.sync()
        stages[name] = round((time.time() - t0) / args.boot_reps * 1e3, 3)
    del w, y, r
    # the refresh's largest kernel class against HBM: its launches in one
    # refresh timed with HIP events, algorithmic bytes from the library
    ctx.profile("ntt_fwd_pass1")
    out = ctx.bootstrap(plan, keys, cts[0])
    prof = ctx.profile_read()
    ctx.profile(None)
    achieved = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] else 0.0
    boot_roof = {"kernel": "ntt_fwd_pass1", "bound": "hbm", "launches": prof["launches"],
                 "avg_launch_us": round(prof["ms"] * 1e3 / max(1, prof["launches"]), 3),
                 "algorithmic_bytes_per_launch": round(prof["bytes"] / max(1, prof["launches"])),
                 "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(achieved / 8000.0, 4)}
    outs = ctx.bootstrap_batch(plan, keys, cts)
    ctx.sync()
    t0 = time.time()
    for _ in range(args.boot_reps):
        outs = ctx.bootstrap_batch(plan, keys, cts)
    ctx.sync()
    batched = (time.time() - t0) / args.boot_reps
    errb = max(float(np.abs(ctx.decrypt(keys, o, z.shape[1]) - z[i]).max()) for i, o in enumerate(outs))
    del outs, out
    # the real-slot refresh of an input at the lowest level it accepts, alone
    # and in the batch
    low = [ctx.mod_drop(c, bs.real_stc) for c in cts]
    rout = ctx.bootstrap(rplan, keys, low[0])
    ctx.sync()
    k0 = ctx.counters()["keyswitches"]
    t0 = time.time()
    for _ in range(args.boot_reps):
        rout = ctx.bootstrap(rplan, keys, low[0])
    ctx.sync()
    rsingle = (time.time() - t0) / args.boot_reps
    rks = (ctx.counters()["keyswitches"] - k0) / args.boot_reps
    routs = ctx.bootstrap_batch(rplan, keys, low)
    ctx.sync()
    t0 = time.time()
    for _ in range(args.boot_reps):
        routs = ctx.bootstrap_batch(rplan, keys, low)
    ctx.sync()
    rbatched = (time.time() - t0) / args.boot_reps
    rerr = max(float(np.abs(ctx.decrypt(keys, o, z.shape[1]) - z[i]).max()) for i, o in enumerate(routs))
    del routs, rout
    # one refresh of one ciphertext replayed from a HIP graph
    # sparse refreshes: one ciphertext and a batch, n-periodic inputs
    sparse = {}
    M = 1 << (bs.logN - 1)
    for name, n, sp in [(str(n), n, sp) for n, sp in splans.items()] + [("%d_real_slots" % n_real, n_real, srplan)]:
        zs = [np.tile(z[i][:n], M // n) for i in range(B)]
        scts = [ctx.encrypt(keys, zs[i], synth.SEED_ENC + 200 + i) for i in range(B)]
        if sp is srplan:
            scts = [ctx.mod_drop(c, bs.real_stc) for c in scts]
        so = ctx.bootstrap(sp, keys, scts[0])
        ctx.sync()
        k0 = ctx.counters()["keyswitches"]
        t0 = time.time()
        for _ in range(args.boot_reps):
            so = ctx.bootstrap(sp, keys, scts[0])
        ctx.sync()
        s1 = (time.time() - t0) / args.boot_reps
        sks = (ctx.counters()["keyswitches"] - k0) / args.boot_reps
        souts = ctx.bootstrap_batch(sp, keys, scts)
        ctx.sync()
        t0 = time.time()
        for _ in range(args.boot_reps):
            souts = ctx.bootstrap_batch(sp, keys, scts)
        ctx.sync()
        sb = (time.time() - t0) / args.boot_reps
        serr = max(float(np.abs(ctx.decrypt(keys, o, M) - zs[i]).max()) for i, o in enumerate(souts))
        sparse[name] = {"ms_per_bootstrap_b1": round(s1 * 1e3, 3), "bootstraps_per_s_b1": round(1.0 / s1, 2),
                          "ms_per_batch": round(sb * 1e3, 3), "bootstraps_per_s_batched": round(B / sb, 2),
                          "keyswitches_per_bootstrap": sks, "max_abs_err": serr}
        del so, souts, scts
    log("bootstrapping: sparse refreshes %s" % sparse)
    graph_ms = {}
    for name, pl, c_in in (("full_slot", plan, cts[0]), ("real_slot", rplan, low[0])):
        g, gouts = ctx.graph_capture_bootstrap(pl, keys, [c_in])
        ctx.sync()
        t0 = time.time()
        for _ in range(args.boot_reps):
            g.launch()
        ctx.sync()
        graph_ms[name] = round((time.time() - t0) / args.boot_reps * 1e3, 3)
        g.free()
        del gouts
    del low
    # the formula KAN with a bootstrapping between layers, with either refresh
    x = synth.inputs(wl, B)
    want = pc.plain_forward(x, layers)
    kin = [ctx.encrypt(keys, x[i], synth.SEED_ENC + 100 + i) for i in range(B)]
    kan = {}
    # (the layer outputs repeat with period 16, so sparse refreshes of 512 and
    # of 64 slots apply)
    for name, pl in (("full_slot_refresh", plan), ("real_slot_refresh", rplan),
                     ("sparse_512_slot_refresh", splans[512]),
                     ("sparse_%d_real_slot_refresh" % n_real, srplan)):
        kout = ctx.eval_kan_boot(model, pl, keys, kin)
        ctx.sync()
        t0 = time.time()
        for _ in range(args.boot_reps):
            kout = ctx.eval_kan_boot(model, pl, keys, kin)
        ctx.sync()
        kan_s = (time.time() - t0) / args.boot_reps
        kerr = max(float(np.abs(ctx.decrypt(keys, o, wl.shape[-1]) - want[i]).max()) for i, o in enumerate(kout))
        kan[name] = {"inferences_per_s": round(B / kan_s, 3), "ms_per_batch": round(kan_s * 1e3, 1),
                     "max_abs_err_vs_fp64_circuit": kerr}
        del kout
    res = {"parameters": "boot16: N=2^16, 51 + 10x45 + 17x58-bit primes, 4 special primes, 4-limb digits, h=192",
           "plan": {"cts_levels": bs.cts, "stc_levels": bs.stc, "K": bs.K, "double_angles": bs.r,
                    "cos_degree": bs.degree, "levels": "%d -> %d" % (bs.L, bs.Lc)},
           "first_call_s": round(first, 3),
           "ms_per_bootstrap_b1": round(single * 1e3, 3),
           "bootstraps_per_s_b1": round(1.0 / single, 2),
           "batch": B, "ms_per_batch": round(batched * 1e3, 3),
           "bootstraps_per_s_batched": round(B / batched, 2),
           "keyswitches_per_bootstrap": ks,
           "stage_ms_b1": stages,
           "roofline_b1": boot_roof,
           "max_abs_err": max(err, errb),
           "real_slots": {"plan": "SlotToCoeff first in %d groups on the input's limbs, one EvalMod" % bs.real_stc,
                          "input_level": bs.real_stc,
                          "ms_per_bootstrap_b1": round(rsingle * 1e3, 3), "bootstraps_per_s_b1": round(1.0 / rsingle, 2),
                          "ms_per_batch": round(rbatched * 1e3, 3), "bootstraps_per_s_batched": round(B / rbatched, 2),
                          "keyswitches_per_bootstrap": rks, "max_abs_err": rerr},
           "sparse_slots": dict(plan="slots = n: SubSum, then %d/%d stage groups over the first log2 n stages; "
                                     "inputs repeat with period n; '_real_slots': SlotToCoeff first in %d groups, "
                                     "the input at level %d" % (bs.cts, bs.stc, bs.real_stc, bs.real_stc), **sparse),
           "graph_replay_ms_b1": graph_ms,
           "kan_formula_with_bootstrapping": dict(
               model="KAN [4,10,10,1], 2 bootstraps per inference, batch %d" % B, **kan)}
    log("bootstrapping:", res)
    del kin, cts, keys, model, plan, rplan
    ctx.close()
    return res


def table3(args):
    """The paper's comparison of the basis approximation with and without
    lazy combination, on one GPU: for each (n_i, g, k) a one-layer KAN
    [n_i, n_o = 10] on U[0,1] inputs, grid [0,1], at the N = 2^16 parameters,
    evaluated for one encrypted input (batch 1, as the paper's latencies)
    (a) in the paper's order (lazy combination: W_f = W'P applied to the
    ColTile bases) and (b) without lazy combination (the bases permuted into
    row order by a homomorphic permutation, then W'); also (c) with the
    restructurings.  Median of `--table3-reps` timed evaluations after a
    warm-up (plaintext caches filled); every variant decrypts within 1e-2 of
    the FP64 circuit."""
    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth
    wl0 = synth.WORKLOADS["image"]
    ctx = hekan.Context(wl0.logN, wl0.L, wl0.scale_bits, wl0.alpha, wl0.w)
    rows = []
    for n_i, g, k in TABLE3_SHAPES:
        wl = synth.Workload("t3", wl0.logN, wl0.L, wl0.scale_bits, wl0.alpha, wl0.w, (n_i, 10), g, k, (0.0, 1.0),
                            31, None, ((7, 7),), 0.05, 0.05, "pixels")
        layers = pc.compile_kan(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024), wl.silu_degree,
                                [list(c) for c in wl.comp_degrees], wl.grid, None, prescale=True)
        x = synth.inputs(wl, 1)[0]
        want = pc.plain_forward(x[None], layers)[0]
        row = {"n_i": n_i, "g": g, "k": k, "n_o": 10}
        for name, flags in (("lazy", hekan.CIRCUIT_PAPER), ("naive", hekan.CIRCUIT_NAIVE_PERMUTATION),
                            ("restructured", hekan.CIRCUIT_RESTRUCTURED)):
            model = ctx.compile(layers, circuit=flags)
            t0 = time.time()
            keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
            ct = ctx.encrypt(keys, x, synth.SEED_ENC)
            out = ctx.eval_kan(model, keys, ct)
            ctx.sync()
            setup = time.time() - t0
            err = float(np.abs(ctx.decrypt(keys, out, 10) - want).max())
            c0 = ctx.counters()
            lat = []
            for _ in range(args.table3_reps):
                t0 = time.perf_counter()
                out = ctx.eval_kan(model, keys, ct)
                ctx.sync()
                lat.append(time.perf_counter() - t0)
            c1 = ctx.counters()
            row[name] = {"ms": round(float(np.median(lat)) * 1e3, 3),
                         "keyswitches": (c1["keyswitches"] - c0["keyswitches"]) // args.table3_reps,
                         "rotation_keys": len(model.rotation_steps()), "max_abs_err_vs_fp64_circuit": err,
                         "setup_s": round(setup, 1)}
            log("table3 %s %s: %s" % ((n_i, g, k), name, row[name]))
            del out, ct, keys, model
        row["speedup_lazy_vs_naive"] = round(row["naive"]["ms"] / row["lazy"]["ms"], 3)
        rows.append(row)
    ctx.close()
    return {"metric": "encrypted KAN layer latency, basis approximation with and without lazy combination",
            "unit": "ms", "n_gpus": 1, "batch": 1, "data": "synthetic",
            "config": {"workload": "one-layer KAN [n_i,10], k, G=g on [0,1], RNS-CKKS N=2^16, L=24, "
                                   "4 special primes, 5-limb digits"}, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16, help="requests per step, split evenly over the engines")
    ap.add_argument("--engines", type=int, default=1,
                    help="contexts (HIP streams, copies of the keys) evaluating parts of the batch concurrently")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="steps of the plain per-ciphertext path (batch 1) timed for comparison; 0 skips")
    ap.add_argument("--workload", default="image")
    ap.add_argument("--graph-steps", type=int, default=10,
                    help="replays of the inference captured into a HIP graph, at the batch and at batch 1 (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-steps", type=int, default=3,
                    help="steps run after the timed region with the roofline kernel's launches timed")
    ap.add_argument("--no-ks-bench", action="store_true", help="skip the key-switch microbenchmark")
    ap.add_argument("--no-word-study", action="store_true",
                    help="skip the integer-words run (every prime on 64-bit integer arithmetic)")
    ap.add_argument("--roofline-kernel", default="ntt_fwd_pass1")
    ap.add_argument("--no-serve", action="store_true", help="skip the continuous-batching server run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default key-switch configuration (fused, spans of 8) at every level")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-saturation", type=int, default=96,
                    help="requests of the serving mix present at once to measure its saturation throughput")
    ap.add_argument("--serve-batch", type=int, default=16)
    ap.add_argument("--native-requests", type=int, default=300,
                    help="Poisson arrivals served by the library's native server (he_submit / he_poll)")
    ap.add_argument("--serve-engines", type=int, default=2,
                    help="serving engines (contexts with their own stream and copy of the keys)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device-to-device copy of this size (counter calibration)")
    ap.add_argument("--no-boot", action="store_true", help="skip the bootstrapping measurement")
    ap.add_argument("--boot-only", action="store_true", help="only the bootstrapping measurement (its own JSON line)")
    ap.add_argument("--boot-profile-plan", choices=("full", "sparse_real"), default="full",
                    help="the refresh --boot-profile repeats: full-slot, or the sparse real-slot one")
    ap.add_argument("--boot-profile", action="store_true",
                    help="with --boot-only: refreshes of one ciphertext separated by 0.2 s idle gaps, for a trace")
    ap.add_argument("--boot-batch", type=int, default=8)
    ap.add_argument("--boot-reps", type=int, default=3)
    ap.add_argument("--table3", action="store_true",
                    help="run only the basis-approximation comparison (lazy combination vs the naive permutation)")
    ap.add_argument("--table3-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): requests are independent, so N GPUs would "
              "serve N queues, each with its own copy of the evaluation keys and no exchange on the "
              "hot path", file=sys.stderr)
        sys.exit(2)

    from paper_2409_07751_amd import compile as pc
    from paper_2409_07751_amd import hekan, synth

    if args.table3:
        print(json.dumps(table3(args)), flush=True)
        return
    if args.boot_only:
        print(json.dumps({"bootstrapping": boot_bench(args)}), flush=True)
        return
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
    B, E = args.batch, args.engines
    if B % E:
        raise SystemExit("--batch must be a multiple of --engines")
    Be = B // E
    x = synth.inputs(wl, B)
    # engines: contexts with their own HIP stream and copy of the evaluation
    # keys (same seed), each evaluating B / E of the requests from its own host
    # thread, so that their kernels overlap on the device
    engines = [(ctx, model, keys)]
    for e in range(1, E):
        c2 = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
        m2 = c2.compile(layers)
        engines.append((c2, m2, c2.keygen(synth.SEED_KEYGEN, steps)))
    parts = [[c.encrypt(k, x[i], synth.SEED_ENC + i) for i in range(e * Be, (e + 1) * Be)]
             for e, (c, m, k) in enumerate(engines)]
    for c, _, _ in engines:
        c.sync()
    cts = parts[0] if E == 1 else [ct for p in parts for ct in p]
    from concurrent.futures import ThreadPoolExecutor
    workers = ThreadPoolExecutor(max_workers=E)

    def run_engine(e):
        c, m, k = engines[e]
        outs = c.eval_kan_batch(m, k, parts[e])
        c.sync()
        return outs

    def step():
        if E == 1:
            return run_engine(0)
        futs = [workers.submit(run_engine, e) for e in range(E)]
        return [o for f in futs for o in f.result()]

    # key-switch configuration per level, chosen by measurement for each
    # engine's batch and for the plain path's batch of one
    tune = {}
    if not args.no_autotune:
        t0 = time.time()
        for nb in sorted({Be, 1}):
            tune[str(nb)] = ctx.autotune(keys, nb)
        for c, _, k in engines[1:]:
            c.autotune(k, Be)
        log("key-switch autotune %.1fs: %s" % (time.time() - t0, tune))

    for w in range(args.warmup):
        t0 = time.time()
        outs = step()
        log("warmup %d: %.3fs" % (w, time.time() - t0))
    # accuracy check of the last warmup output against the plain FP64 circuit
    want = pc.plain_forward(x, layers)
    err = max(float(np.abs(engines[i // Be][0].decrypt(engines[i // Be][2], outs[i], wl.shape[-1]) - want[i]).max())
              for i in range(B))
    log("max |decrypt - fp64 circuit| = %.3e" % err)
    del outs

    def counters():
        cs = [c.counters() for c, _, _ in engines]
        return {k: sum(v[k] for v in cs) for k in cs[0]}

    # the timed steps: no kernel timer (no events between launches)
    c0 = counters()
    lat = []
    for c, _, _ in engines:
        c.sync()
    t_start = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        outs = step()
        lat.append(time.perf_counter() - t0)
        del outs
    for c, _, _ in engines:
        c.sync()
    elapsed = time.perf_counter() - t_start
    c1 = counters()
    # the roofline's kernel timing in separate steps after the timed ones, on
    # engine 0 alone (its batch of B / E)
    ctx.profile(args.roofline_kernel)
    for s in range(args.roofline_steps):
        del_outs = run_engine(0)
        del del_outs
    prof = ctx.profile_read()
    ctx.profile(None)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    roof = roofline(args.roofline_kernel, prof, Be)
    if roof is not None:
        roof["timed_in"] = "%d separate steps after the timed region (HIP events around each launch)" % \
            args.roofline_steps
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
                               "5-limb digits", "batch": B, "engines": E, "batch_per_engine": Be,
                   "levels": wl.L, "log_n": wl.logN},
        "keyswitches_per_s": round(ks_per_step * args.steps / elapsed, 1),
        "keyswitches_per_inference": ks_per_step / B,
        "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
        "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3),
        "latency": "per timed step (one batch of all requests; per-request latency: serving)",
        "max_abs_err_vs_fp64_circuit": err,
        "launches_per_step": (c1["launches"] - c0["launches"]) / args.steps,
        "roofline": roof,
        "keyswitch_autotune": tune or None,
    }
    if args.plain_steps:
        res["plain_path"] = plain_path(ctx, model, keys, cts[0], args.plain_steps)
        res["batched_vs_plain"] = round(res["value"] / res["plain_path"]["inferences_per_s"], 3)
    if not args.no_ks_bench:
        res["keyswitch_bench"] = ks_bench(ctx, keys, wl, steps)
    if args.graph_steps:
        res["graph_path"] = [graph_path(ctx, model, keys, c, args.graph_steps, want, wl.shape[-1])
                             for c in (parts[0], parts[0][:1])]
    if not args.no_serve:
        res["serving"], res["batched_mix"] = serve_run(args)
    if not args.no_word_study:
        res["word_size_study"] = word_study(args, layers, wl, x, want)
        log("word-size study:", res["word_size_study"])
    res["silu_fit_comparison"] = silu_fits()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl)
    workers.shutdown()
    del cts, parts, keys, model
    for c, _, _ in engines[1:]:
        c.close()
    del engines
    ctx.close()
    if not args.no_boot:
        res["bootstrapping"] = boot_bench(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
