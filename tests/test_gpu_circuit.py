"""The layer circuit in the paper's order and with each restructuring, on the
GPU through the C ABI, bit-exact against the oracle's circuit with the same
options (he_kan_desc.circuit <-> oracle.circuit.Circuit).

The paper's order is Algorithm 2 with both PolyComps and the two linear
layers of the Lazy Combination section as two products, each folded over all
slots; the toy workload (g = 2, k = 1, the grid of the paper's example of the
basis construction) has g+2k = 4 repeat-packed copies, one block short of the
five a shared second comparison needs, so its first layer takes Algorithm 2's
two-PolyComp branch with every option."""
import sys

import numpy as np
import pytest

from oracle import ckks as O
from oracle import circuit, kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu

# he_kan_desc.circuit bits: 1 shared comparison, 2 fused linear layers, 4 folded period,
# 8 no lazy combination (the naive permutation)
VARIANTS = [0, 1, 2, 4, 16, 23]


def note(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def oracle_circuit(flags):
    return circuit.Circuit(bool(flags & 1), bool(flags & 2), bool(flags & 4), bool(flags & 8), bool(flags & 16))


def model_layers(wl):
    nl = len(wl.shape) - 1
    return kan.compile_model(synth.raw_weights(wl), synth.calibration_inputs(wl), [wl.silu_degree] * nl,
                             [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)


@pytest.fixture(scope="module")
def hk():
    from paper_2409_07751_amd import hekan
    return hekan


def run_variants(hk, name, variants):
    """Every variant of the workload's model, layer by layer with the
    client-aided refresh: residues equal the oracle's, rotation steps agree,
    and the decrypted output is within 1e-2 of the FP64 circuit."""
    wl = synth.WORKLOADS[name]
    layers = model_layers(wl)
    ctx = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
    try:
        models = {f: ctx.compile(layers, refresh=True, circuit=f) for f in variants}
        for f, m in models.items():
            assert m.rotation_steps() == circuit.rotation_steps(layers, octx.p.slots, circ=oracle_circuit(f)), f
        steps = sorted(set(s for m in models.values() for s in m.rotation_steps()))
        note(name, "keygen", len(steps))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
        x = synth.inputs(wl, 1)[0]
        want = kan.he_friendly_kan(x[None], layers)[0]
        for f, model in models.items():
            circ = oracle_circuit(f)
            ct = ctx.encrypt(keys, x, synth.SEED_ENC)
            oct_ = ev.encrypt(x, synth.SEED_ENC)
            n_blk = layers[0].n_in
            for li, L in enumerate(layers):
                note(name, "circuit", f, "layer", li)
                out = ctx.eval_kan_layer(model, keys, li, ct)
                oout, n_blk = circuit.layer_forward(ev, [oct_], L, n_blk, li == 0, circ=circ)
                e = out.export()
                assert out.level == oout.level, (f, li)
                assert (e[0] == oout.c0).all() and (e[1] == oout.c1).all(), "circuit %d layer %d residues" % (f, li)
                if li + 1 < len(layers):
                    v = ev.decrypt(oout, octx.p.slots)
                    ct = ctx.encrypt(keys, v, 100 + li)
                    oct_ = ev.encrypt(v, 100 + li)
            y = ctx.decrypt(keys, out, layers[-1].n_out)
            note(name, "circuit", f, "max err", np.abs(y - want).max())
            assert np.abs(y - want).max() < 1e-2
    finally:
        ctx.close()


def test_tiny_paper_order_and_each_restructuring_bit_exact(hk):
    run_variants(hk, "tiny", VARIANTS)


def test_toy_two_polycomp_branch_bit_exact(hk):
    wl = synth.WORKLOADS["toy"]
    # the first layer cannot share the comparison: 4 copies < g+2k+1 = 5 blocks
    assert (1 << (wl.g + 2 * wl.k - 1).bit_length()) < wl.g + 2 * wl.k + 1
    run_variants(hk, "toy", [0, 23])


def test_toy_without_lazy_combination_bit_exact(hk):
    """The comparison method of the paper's basis experiments (bit 8: the
    bases permuted into row order by a homomorphic permutation, then W'),
    alone and with the shared comparison, bit-exact against the oracle."""
    run_variants(hk, "toy", [8, 9])
