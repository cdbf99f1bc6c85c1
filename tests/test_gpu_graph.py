"""A batched inference captured into a HIP graph (he_graph_*): every replay,
with eager work of the same context between replays, reproduces the eager
result bit for bit."""
import sys

import numpy as np
import pytest

from oracle import kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny_setup():
    from paper_2409_07751_amd import hekan
    wl = synth.WORKLOADS["tiny"]
    raw = synth.raw_weights(wl)
    layers = kan.compile_model(raw, synth.calibration_inputs(wl), [wl.silu_degree] * 2,
                               [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    note("tiny context")
    ctx = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    model = ctx.compile(layers[:1])
    keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
    yield wl, ctx, model, keys
    ctx.close()


@pytest.mark.parametrize("n", [3, 1])
def test_graph_replays_equal_eager(tiny_setup, n):
    wl, ctx, model, keys = tiny_setup
    xs = synth.inputs(wl, n, stream=11)
    cts = [ctx.encrypt(keys, xs[i], 70 + i) for i in range(n)]
    eager = [o.export() for o in ctx.eval_kan_batch(model, keys, cts)]
    note("capture, batch", n)
    graph, outs = ctx.capture_kan_batch(model, keys, cts)
    ctx.sync()
    for i in range(n):
        assert (outs[i].export() == eager[i]).all(), "captured run, request %d" % i
    for rep in range(3):
        # eager work of the same context between replays (allocates and frees pool buffers)
        other = ctx.eval_kan_batch(model, keys, cts[::-1])
        graph.launch()
        ctx.sync()
        for i in range(n):
            assert (outs[i].export() == eager[i]).all(), "replay %d, request %d" % (rep, i)
            assert (other[n - 1 - i].export() == eager[i]).all(), "eager run between replays"
        note("replay", rep, "ok")
    graph.free()
    assert (outs[0].export() == eager[0]).all()
    y = ctx.decrypt(keys, outs[0], wl.shape[1])
    assert np.isfinite(y).all()


@pytest.mark.timeout(900)
def test_graph_image_model_bit_exact():
    """The full [784,64,10] inference at N = 2^16 (both layers) captured for a
    batch of two: replays, with eager work between them, equal the eager
    result residue for residue and decrypt within 1e-2 of the FP64 circuit."""
    from paper_2409_07751_amd import hekan
    wl = synth.WORKLOADS["image"]
    raw = synth.raw_weights(wl)
    layers = kan.compile_model(raw, synth.calibration_inputs(wl, 1024), [wl.silu_degree] * 2,
                               [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    note("image context")
    ctx = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        model = ctx.compile(layers)
        keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
        xs = synth.inputs(wl, 2, stream=13)
        cts = [ctx.encrypt(keys, xs[i], 80 + i) for i in range(2)]
        eager = [o.export() for o in ctx.eval_kan_batch(model, keys, cts)]
        note("image capture, batch 2")
        graph, outs = ctx.capture_kan_batch(model, keys, cts)
        for rep in range(2):
            ctx.eval_kan(model, keys, cts[1])
            graph.launch()
            ctx.sync()
            for i in range(2):
                assert (outs[i].export() == eager[i]).all(), "replay %d, request %d" % (rep, i)
            note("image replay", rep, "ok")
        want = kan.he_friendly_kan(xs, layers)
        for i in range(2):
            assert np.abs(ctx.decrypt(keys, outs[i], 10) - want[i]).max() < 1e-2
        graph.free()
    finally:
        ctx.close()
