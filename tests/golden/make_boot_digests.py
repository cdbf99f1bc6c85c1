"""Write tests/golden/boot_digests.json: digests of the oracle's residues for
one CKKS bootstrapping on the N = 2^16 bootstrappable parameter set (boot16 of
paper_2409_07751_amd.synth: 51 + 10x45 + 17x58-bit primes, 4 special primes,
4-limb digits, sparse secret of weight 192), which the GPU parity tests
compare against; and the same for the real-slot refresh with SlotToCoeff
first (`real`), and the sparsely packed refresh of 512 slots of a 512-periodic
input (`sparse512`; `--sparse-only` adds just that entry to the existing file).

Runs only the CPU oracle (oracle/) on seeded synthetic inputs; nothing here
touches the GPU path.  The input is synth.boot_inputs(boot16, 1)[0]
encrypted with seed SEED_ENC at the top computation level (keys from
SEED_KEYGEN with the bootstrapping's rotation steps).  For the input and
every stage output (CoeffToSlot, the two EvalMod results, the recombined
ciphertext, the refreshed output) it stores the level, the SHA-256 of the
coefficient-form residues as the little-endian uint64 array [2][level+1][N]
(c0 then c1, limb-major) and a few sampled residues for diagnosis, plus the
largest decrypted error of the output against the input.  Takes a few
minutes.

    python tests/golden/make_boot_digests.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import boot, ckks as O  # noqa: E402
from paper_2409_07751_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "boot_digests.json")
SAMPLES = [(0, 0, 0), (1, 0, 12345), (0, 1, 65535), (1, 2, 4096), (0, 5, 31337), (1, 7, 77)]


def entry(ct):
    a = np.ascontiguousarray(np.stack([ct.c0, ct.c1]).astype("<u8"))
    pos = [(p, l % (ct.level + 1), n) for p, l, n in SAMPLES]
    return {"level": int(ct.level), "sha256": hashlib.sha256(a.tobytes()).hexdigest(), "positions": pos,
            "sampled": [int((ct.c0, ct.c1)[p][l][n]) for p, l, n in pos]}


SPARSE_SLOTS = 512


def sparse_input(bs):
    """the first 512 values of synth.boot_inputs(boot16, 1)[0], repeated over
    every slot"""
    z = synth.boot_inputs(bs, 1)[0]
    return np.tile(z[:SPARSE_SLOTS], len(z) // SPARSE_SLOTS)


def sparse_entry(bs, p, ctx):
    sbp = boot.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree, slots=SPARSE_SLOTS)
    steps = boot.rotation_steps(bs.logN, sbp)
    ev = O.Oracle(ctx, O.Keys(ctx, synth.SEED_KEYGEN, steps))
    ct = ev.encrypt(sparse_input(bs), synth.SEED_ENC)
    tr = {}
    t0 = time.time()
    out = boot.bootstrap(ev, ct, sbp, tr)
    print("sparse bootstrap %.0f s, %s" % (time.time() - t0, ev.count), flush=True)
    err = float(np.abs(ev.decrypt(out, p.slots) - ev.decrypt(ct, p.slots)).max())
    print("sparse: max |decrypt(out) - decrypt(in)| = %.3g" % err, flush=True)
    return {"plan": "slots %d: SubSum, CoeffToSlot and SlotToCoeff in %d/%d groups over the first %d stages"
                    % (SPARSE_SLOTS, bs.cts, bs.stc, SPARSE_SLOTS.bit_length() - 1),
            "input": "the first %d values of synth.boot_inputs(boot16, 1)[0] repeated, encrypted with seed SEED_ENC"
                     % SPARSE_SLOTS,
            "steps": steps, "max_abs_err": err,
            "stages": {"input": entry(ct), "cts": entry(tr["cts"]), "output": entry(out)}}


def main():
    bs = synth.BOOTSETS["boot16"]
    if "--sparse-only" in sys.argv:
        p = O.Params(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, bs.base_bits, bs.special_bits, bs.sigma,
                     bs.boot_levels, bs.boot_bits, bs.h)
        res = json.load(open(OUT))
        res["sparse512"] = sparse_entry(bs, p, O.Context(p))
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)
        print("wrote", OUT, flush=True)
        return
    p = O.Params(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, bs.base_bits, bs.special_bits, bs.sigma,
                 bs.boot_levels, bs.boot_bits, bs.h)
    ctx = O.Context(p)
    bp = boot.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)
    steps = boot.rotation_steps(bs.logN, bp)
    rbp = boot.make_params(bs.cts, bs.real_stc, bs.K, bs.r, bs.degree, real_slots=True)
    rsteps = boot.rotation_steps(bs.logN, rbp)
    t0 = time.time()
    ev = O.Oracle(ctx, O.Keys(ctx, synth.SEED_KEYGEN, sorted(set(steps) | set(rsteps))))
    print("keygen %.0f s (%d keys)" % (time.time() - t0, len(steps)), flush=True)
    z = synth.boot_inputs(bs, 1)[0]
    ct = ev.encrypt(z, synth.SEED_ENC)
    tr = {}
    t0 = time.time()
    out = boot.bootstrap(ev, ct, bp, tr)
    print("bootstrap %.0f s, %s" % (time.time() - t0, ev.count), flush=True)
    err = float(np.abs(ev.decrypt(out, p.slots) - ev.decrypt(ct, p.slots)).max())
    res = {"workload": "boot16: N=2^16, 51 + 10x45 + 17x58-bit primes, 4 special primes, 4-limb digits, h=192; "
                       "CoeffToSlot and SlotToCoeff in %d/%d groups, EvalMod K=%g, r=%d, degree %d"
                       % (bs.cts, bs.stc, bs.K, bs.r, bs.degree),
           "input": "synth.boot_inputs(boot16, 1)[0] encrypted with seed SEED_ENC at the top computation level",
           "steps": steps, "max_abs_err": err,
           "stages": {"input": entry(ct), "cts": entry(tr["cts"]), "evalmod_lo": entry(tr["evalmod"][0]),
                      "evalmod_hi": entry(tr["evalmod"][1]), "recombined": entry(tr["recombined"]),
                      "output": entry(out)}}
    # the real-slot refresh (SlotToCoeff first) of the same input
    tr = {}
    t0 = time.time()
    rout = boot.bootstrap(ev, ct, rbp, tr)
    print("real-slot bootstrap %.0f s" % (time.time() - t0), flush=True)
    rerr = float(np.abs(ev.decrypt(rout, p.slots) - ev.decrypt(ct, p.slots)).max())
    res["real"] = {"plan": "SlotToCoeff first in %d groups, CoeffToSlot in %d, one EvalMod (K=%g, r=%d, degree %d)"
                           % (bs.real_stc, bs.cts, bs.K, bs.r, bs.degree),
                   "steps": rsteps, "max_abs_err": rerr,
                   "stages": {"stc_first": entry(tr["stc_first"]), "cts": entry(tr["cts"]),
                              "evalmod": entry(tr["evalmod"]), "output": entry(rout)}}
    print("real-slot: max |decrypt(out) - decrypt(in)| = %.3g" % rerr, flush=True)
    res["sparse512"] = sparse_entry(bs, p, ctx)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("max |decrypt(out) - decrypt(in)| = %.3g; wrote %s" % (err, OUT), flush=True)


if __name__ == "__main__":
    main()
