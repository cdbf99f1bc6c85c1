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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--workload", default="image")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every box in this setup has a single MI355X "
              "(requests shard across GPUs with no exchange on the hot path; see DESIGN.md)", file=sys.stderr)
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
    t_start = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        outs = step()
        lat.append(time.perf_counter() - t0)
        del outs
    ctx.sync()
    elapsed = time.perf_counter() - t_start
    c1 = ctx.counters()
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
    }
    del cts, keys, model
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
