"""Several input vectors in one ciphertext (feature i of vector s in slot
i S + s) on the GPU: layer residues equal the oracle's bit for bit, and every
vector's decrypted output is within 1e-2 of the FP64 HE-friendly circuit.
All GPU work goes through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import ckks as O
from oracle import circuit, kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-packed]", *a, flush=True)
    sys.stdout.flush()


def compiled(wl, ncal=1024):
    raw = synth.raw_weights(wl)
    return kan.compile_model(raw, synth.calibration_inputs(wl, ncal), [wl.silu_degree] * len(raw),
                             [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)


def context(wl):
    from paper_2409_07751_amd import hekan
    return hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)


def test_tiny_32_vectors_bit_exact():
    """[2,5,1] at N = 2^13 with 32 vectors per ciphertext and the client-aided
    refresh between layers: both layers' residues equal the oracle's, and all
    32 outputs are within 1e-2 of the FP64 circuit."""
    wl = synth.WORKLOADS["tiny"]
    S = 32
    layers = compiled(wl, 4096)
    ctx = context(wl)
    try:
        octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
        model = ctx.compile(layers, refresh=True, samples=S)
        steps = model.rotation_steps()
        assert steps == circuit.rotation_steps(layers, octx.p.slots, S, circuit.RESTRUCTURED)
        note("keygen", len(steps))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
        X = synth.inputs(wl, S)
        ct = ctx.encrypt_input(model, keys, X, synth.SEED_ENC)
        oct_ = ev.encrypt(circuit.pack_samples(X, S), synth.SEED_ENC)
        n_blk = 0
        for li, L in enumerate(layers):
            note("layer", li)
            out = ctx.eval_kan_layer(model, keys, li, ct)
            oout, n_blk = circuit.layer_forward(ev, [oct_], L, n_blk, li == 0, S, circuit.RESTRUCTURED)
            e = out.export()
            assert out.level == oout.level
            assert (e[0] == oout.c0).all() and (e[1] == oout.c1).all(), "layer %d residues differ" % li
            if li + 1 < len(layers):
                v = ev.decrypt(oout, octx.p.slots)
                ct = ctx.encrypt(keys, v, 100 + li)
                oct_ = ev.encrypt(v, 100 + li)
        Y = ctx.decrypt_output(model, keys, out, 1)
        want = kan.he_friendly_kan(X, layers)
        assert np.abs(Y - want).max() < 1e-2
    finally:
        ctx.close()


@pytest.mark.timeout(900)
def test_formula_256_vectors_per_request():
    """[4,10,10,1] at N = 2^15 (16 levels, client-aided refresh between the
    three layers) on 256 input vectors: 4 ciphertexts of 64 vectors (64 x 16
    repeat-packed blocks of 4 features fill the 16384 slots of layer 1; the
    hidden layers need 16 blocks of 16 x 64 slots), run as one batch; every
    one of the 256 outputs is within 1e-2 of the FP64 circuit, and the
    batch gives the same residues as a ciphertext alone."""
    wl = synth.WORKLOADS["formula"]
    S = 64
    layers = compiled(wl)
    ctx = context(wl)
    try:
        model = ctx.compile(layers, refresh=True, samples=S)
        steps = model.rotation_steps()
        assert steps == circuit.rotation_steps(layers, 1 << (wl.logN - 1), S, circuit.RESTRUCTURED)
        note("formula keygen", len(steps))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        X = synth.inputs(wl, 256)
        cts = [ctx.encrypt_input(model, keys, X[64 * j:64 * (j + 1)], synth.SEED_ENC + j) for j in range(4)]
        alone = ctx.eval_kan_layer(model, keys, 0, cts[2])
        for li in range(len(layers)):
            note("formula layer", li)
            outs = ctx.eval_kan_layer_batch(model, keys, li, cts)
            if li == 0:
                assert (outs[2].export() == alone.export()).all()
            if li + 1 < len(layers):
                # client-aided refresh: decrypt, re-encrypt at the top level
                cts = [ctx.encrypt(keys, ctx.decrypt(keys, o, ctx.slots), 200 + 10 * li + j)
                       for j, o in enumerate(outs)]
        Y = np.concatenate([ctx.decrypt_output(model, keys, o, 1) for o in outs])
        want = kan.he_friendly_kan(X, layers)
        note("max err", np.abs(Y - want).max())
        assert np.abs(Y - want).max() < 1e-2
    finally:
        ctx.close()


@pytest.mark.timeout(900)
def test_formula_layers_bit_exact():
    """[4,10,10,1] at N = 2^15 (17 Q limbs, 2 special primes, 2-limb digits)
    on one ciphertext of 64 vectors, layer by layer with the client-aided
    refresh: every layer's residues equal the oracle's (the two-PolyComp
    branch of Algorithm 2 on the 16 repeat-packed copies, the degree-7
    composite stages, the degree-27 SiLU series, the N = 2^15 transforms),
    with the default restructurings; the first layer in the paper's order
    too."""
    from paper_2409_07751_amd import hekan
    wl = synth.WORKLOADS["formula"]
    S = 64
    layers = compiled(wl)
    ctx = context(wl)
    try:
        octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
        model = ctx.compile(layers, refresh=True, samples=S)
        paper = ctx.compile(layers, refresh=True, samples=S, circuit=hekan.CIRCUIT_PAPER)
        steps = sorted(set(model.rotation_steps()) | set(paper.rotation_steps()))
        assert paper.rotation_steps() == circuit.rotation_steps(layers, octx.p.slots, S, circuit.PAPER)
        note("formula keygen", len(steps))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
        X = synth.inputs(wl, 256)[:S]
        x = circuit.pack_samples(X, S)
        ct = ctx.encrypt(keys, x, synth.SEED_ENC)
        oct_ = ev.encrypt(x, synth.SEED_ENC)
        assert (ct.export() == np.stack([oct_.c0, oct_.c1])).all()
        note("formula layer 0, paper order")
        out = ctx.eval_kan_layer(paper, keys, 0, ct)
        oout, _ = circuit.layer_forward(ev, [oct_], layers[0], 0, True, S, circuit.PAPER)
        e = out.export()
        assert out.level == oout.level
        assert (e[0] == oout.c0).all() and (e[1] == oout.c1).all(), "paper-order layer 0 residues differ"
        n_blk = 0
        for li, L in enumerate(layers):
            note("formula layer", li)
            out = ctx.eval_kan_layer(model, keys, li, ct)
            oout, n_blk = circuit.layer_forward(ev, [oct_], L, n_blk, li == 0, S, circuit.RESTRUCTURED)
            e = out.export()
            assert out.level == oout.level
            assert (e[0] == oout.c0).all() and (e[1] == oout.c1).all(), "layer %d residues differ" % li
            if li + 1 < len(layers):
                v = ev.decrypt(oout, octx.p.slots)
                ct = ctx.encrypt(keys, v, 300 + li)
                oct_ = ev.encrypt(v, 300 + li)
        Y = ctx.decrypt_output(model, keys, out, 1)
        assert np.abs(Y - kan.he_friendly_kan(X, layers)).max() < 1e-2
    finally:
        ctx.close()
