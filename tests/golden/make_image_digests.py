"""Write tests/golden/image_digests.json: digests of the oracle's residues for
the encrypted [784,64,10] inference at N = 2^16 (25 Q limbs, 4 special primes,
5-limb digits), and for the first layer of [3072,128,10] at the same
parameters (`--cifar`), which the GPU parity tests compare against.

Runs only the CPU oracle (oracle/) on the seeded synthetic inputs of
paper_2409_07751_amd.synth; nothing here touches the GPU path.  For each
circuit (the paper's order and every restructuring) and each layer output it
stores the level, the SHA-256 of the coefficient-form residues as the
little-endian uint64 array [2][level+1][N] (c0 then c1, limb-major), and a
few sampled residues for diagnosis.  Takes a few minutes per circuit.

    python tests/golden/make_image_digests.py [--circuits paper,restructured]
    python tests/golden/make_image_digests.py --cifar
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ckks as O, circuit, kan  # noqa: E402
from paper_2409_07751_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "image_digests.json")
CIRCUITS = {"paper": circuit.PAPER, "restructured": circuit.RESTRUCTURED}
# sampled (component, limb, coefficient) positions (limb taken modulo the limb count)
SAMPLES = [(0, 0, 0), (0, 0, 1), (1, 0, 12345), (0, 1, 65535), (1, 2, 4096), (0, 5, 31337), (1, 7, 77)]


def digest(ct):
    a = np.ascontiguousarray(np.stack([ct.c0, ct.c1]).astype("<u8"))
    return hashlib.sha256(a.tobytes()).hexdigest()


def image_layers(wl):
    return kan.compile_model(synth.raw_weights(wl), synth.calibration_inputs(wl, 1024), [wl.silu_degree] * 2,
                             [list(c) for c in wl.comp_degrees], wl.grid, prescale=wl.prescale)


def cifar_first_layer(res):
    """The [3072,128,10] model's first layer at the same parameters, restructured: its input in two
    ciphertexts (features [0, 2048) and [2048, 3072), encrypted with seeds SEED_ENC and SEED_ENC + 1),
    both chunks packed, expanded and multiplied by their columns, summed and folded."""
    wl = synth.WORKLOADS["cifar"]
    layers = image_layers(wl)
    octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
    circ = circuit.RESTRUCTURED
    steps = circuit.rotation_steps(layers[:1], octx.p.slots, circ=circ)
    ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
    x = synth.inputs(wl, 1)[0]
    bounds = circuit.chunk_bounds(layers[0], octx.p.slots)
    cts = [ev.encrypt(x[lo:hi], synth.SEED_ENC + c) for c, (lo, hi) in enumerate(zip(bounds[:-1], bounds[1:]))]
    t0 = time.time()
    ct, _ = circuit.layer_forward(ev, cts, layers[0], 0, True, circ=circ)
    pos = [(p, l % (ct.level + 1), n) for p, l, n in SAMPLES]
    res["cifar"] = {"workload": "cifar: KAN [3072,128,10], first layer, N=2^16, L=24, 4 special primes, 5-limb digits",
                    "input": "synth.inputs(cifar, 1)[0] in chunks %s, chunk c encrypted with seed SEED_ENC + c" % bounds,
                    "restructured": {"steps": steps, "bounds": bounds,
                                     "layers": [{"level": int(ct.level), "sha256": digest(ct), "positions": pos,
                                                 "sampled": [int((ct.c0, ct.c1)[p][l][n]) for p, l, n in pos]}]}}
    print("cifar first layer: level %d in %.0f s" % (ct.level, time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--circuits", default="paper,restructured")
    ap.add_argument("--cifar", action="store_true", help="only (re)write the [3072,128,10] first-layer digest")
    args = ap.parse_args()
    if args.cifar:
        res = json.load(open(OUT))
        cifar_first_layer(res)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)
        print("wrote", OUT)
        return
    wl = synth.WORKLOADS["image"]
    layers = image_layers(wl)
    octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    res["workload"] = "image: KAN [784,64,10], N=2^16, L=24, 4 special primes, 5-limb digits"
    res["input"] = "synth.inputs(image, 1)[0], encrypted with seed SEED_ENC; keys seed SEED_KEYGEN"
    x = synth.inputs(wl, 1)[0]
    for name in args.circuits.split(","):
        circ = CIRCUITS[name]
        steps = circuit.rotation_steps(layers, octx.p.slots, circ=circ)
        t0 = time.time()
        ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
        print("%s: keys for %d steps in %.0f s" % (name, len(steps), time.time() - t0), flush=True)
        ct = ev.encrypt(x, synth.SEED_ENC)
        outs = []
        n_blk = 0
        for li, L in enumerate(layers):
            t0 = time.time()
            ct, n_blk = circuit.layer_forward(ev, [ct], L, n_blk, li == 0, circ=circ)
            pos = [(p, l % (ct.level + 1), n) for p, l, n in SAMPLES]
            outs.append({"level": int(ct.level), "sha256": digest(ct), "positions": pos,
                         "sampled": [int((ct.c0, ct.c1)[p][l][n]) for p, l, n in pos]})
            print("%s layer %d: level %d in %.0f s" % (name, li, ct.level, time.time() - t0), flush=True)
        res[name] = {"steps": steps, "layers": outs}
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
