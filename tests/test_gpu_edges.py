"""Edge cases and error paths of the C ABI on the GPU: empty batches,
arguments the library must reject with an error code (never a fault), handles
of another context, a layer deeper than its input's levels.  The rejected
arguments are caught on the host before a kernel is launched for them; the
too-deep layer stops at the first step that would go below level 0."""
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
def hk():
    from paper_2409_07751_amd import hekan
    return hekan


@pytest.fixture(scope="module")
def tiny(hk):
    wl = synth.WORKLOADS["tiny"]
    raw = synth.raw_weights(wl)
    layers = kan.compile_model(raw, synth.calibration_inputs(wl), [wl.silu_degree] * 2,
                               [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    note("tiny context")
    ctx = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    model = ctx.compile(layers[:1])
    keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
    yield wl, layers, ctx, model, keys
    ctx.close()


def raises(hk, code, fn, *a):
    with pytest.raises(hk.HeError) as e:
        fn(*a)
    assert e.value.code == code, str(e.value)
    return e.value


def test_empty_batches(hk, tiny):
    wl, layers, ctx, model, keys = tiny
    note("empty batches")
    assert ctx.eval_kan_batch(model, keys, []) == []
    raises(hk, hk.HE_EINVAL, ctx.capture_kan_batch, model, keys, [])
    # the context still works afterwards
    x = synth.inputs(wl, 1, stream=3)[0]
    ct = ctx.encrypt(keys, x, 5)
    assert len(ctx.eval_kan_batch(model, keys, [ct])) == 1


def test_rejected_arguments(hk, tiny):
    wl, layers, ctx, model, keys = tiny
    x = synth.inputs(wl, 2, stream=4)
    a, b = ctx.encrypt(keys, x[0], 6), ctx.encrypt(keys, x[1], 7)
    low = ctx.rescale(b)
    note("rejected arguments")
    raises(hk, hk.HE_EINVAL, ctx.add, a, low)                        # levels differ
    raises(hk, hk.HE_EINVAL, ctx.eval_kan_batch, model, keys, [a, low])   # batch of mixed levels
    have = {int(v) % ctx.slots for v in model.rotation_steps()}
    miss = next(v for v in range(1, ctx.slots) if v not in have)
    raises(hk, hk.HE_EKEY, ctx.rotate, keys, a, miss)                # no key for this step
    raises(hk, hk.HE_EKEY, ctx.rotate_sum, keys, [a, a], [0, miss])  # no key for one of the steps
    raises(hk, hk.HE_ESHAPE, ctx.rotate_sum, keys, [a, low], [0, 1])  # levels differ
    raises(hk, hk.HE_EINVAL, ctx.rotate_sum, keys, [], [])           # no terms
    raises(hk, hk.HE_EINVAL, ctx.decrypt, keys, a, ctx.slots + 1)    # more values than slots
    raises(hk, hk.HE_ESHAPE, ctx.encrypt, keys, np.zeros(ctx.slots + 1), 1)
    q, _, _ = ctx.primes()
    res = a.export()
    res[1, 0, 17] = q[0]                                              # a residue not reduced
    raises(hk, hk.HE_EINVAL, ctx.import_ct, res, wl.L)
    raises(hk, hk.HE_EINVAL, ctx.eval_kan_layer, model, keys, 1, a)  # layer out of range
    # a model compiled with a refresh between layers runs layer by layer only
    two = ctx.compile(layers, refresh=True)
    raises(hk, hk.HE_ESTATE, ctx.eval_kan, two, keys, a)


def test_handles_of_another_context(hk, tiny):
    """Keys and ciphertexts of another context are refused with HE_ESTATE by
    every entry point that takes them, before any kernel runs: a context of
    the same size (the same seeds give the same ciphertext there) and one of
    a different size (N = 2^12, other limb counts), whose keys a kernel of
    this context must never read."""
    wl, layers, ctx, model, keys = tiny
    same = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    small = hk.Context(12, 3, 30, 1, 1)
    try:
        x = synth.inputs(wl, 1)[0]
        mine = ctx.encrypt(keys, x, 9)
        ok = same.keygen(synth.SEED_KEYGEN, [])
        ct = same.encrypt(ok, x, 9)
        assert (ct.export() == mine.export()).all()
        sk = small.keygen(synth.SEED_KEYGEN, [1])
        sct = small.encrypt(sk, x, 9)
        for other_keys, other_ct in ((ok, ct), (sk, sct)):
            note("handles of another context", other_ct.ctx.N)
            raises(hk, hk.HE_ESTATE, ctx.eval_kan, model, keys, other_ct)           # ciphertext
            raises(hk, hk.HE_ESTATE, ctx.eval_kan, model, other_keys, mine)         # evaluation keys
            raises(hk, hk.HE_ESTATE, ctx.eval_kan_batch, model, other_keys, [mine])
            raises(hk, hk.HE_ESTATE, ctx.eval_kan_layer, model, other_keys, 0, mine)
            raises(hk, hk.HE_ESTATE, ctx.eval_kan_layer_batch, model, other_keys, 0, [mine])
            raises(hk, hk.HE_ESTATE, ctx.capture_kan_batch, model, other_keys, [mine])
            raises(hk, hk.HE_ESTATE, ctx.encrypt, other_keys, x, 1)                 # secret key
            raises(hk, hk.HE_ESTATE, ctx.decrypt, other_keys, mine, 4)
            raises(hk, hk.HE_ESTATE, ctx.decrypt, keys, other_ct, 4)
            raises(hk, hk.HE_ESTATE, ctx.mul, other_keys, mine, mine)
            raises(hk, hk.HE_ESTATE, ctx.mul, keys, mine, other_ct)
            raises(hk, hk.HE_ESTATE, ctx.rotate, other_keys, mine, 1)
            raises(hk, hk.HE_ESTATE, ctx.rotate, keys, other_ct, 1)
            raises(hk, hk.HE_ESTATE, ctx.rotate_sum, other_keys, [mine, mine], [0, 1])
            raises(hk, hk.HE_ESTATE, ctx.rotate_sum, keys, [mine, other_ct], [0, 1])
            raises(hk, hk.HE_ESTATE, ctx.add, mine, other_ct)
            raises(hk, hk.HE_ESTATE, ctx.rescale, other_ct)
            raises(hk, hk.HE_ESTATE, ctx.lincomb, [mine, other_ct], [1.0, 2.0], 3)
            raises(hk, hk.HE_ESTATE, ctx.autotune, other_keys, 1)
            c = ctx
            with pytest.raises(hk.HeError) as e:
                c.check(c.lib.he_eval_keys_export(c.h, other_keys.ek.h, 0, 0, hk._ptr(np.zeros(1, np.uint64)), 1))
            assert e.value.code == hk.HE_ESTATE
        # the context is still usable and exact
        assert (ctx.rotate(keys, mine, 1).export() == ctx.rotate(keys, mine, 1).export()).all()
    finally:
        same.close()
        small.close()


def test_handles_outlive_their_context(hk):
    """Handles may be freed after he_ctx_destroy: the library releases the
    context's device memory when the last handle made from it goes."""
    wl = synth.WORKLOADS["tiny"]
    c = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    keys = c.keygen(synth.SEED_KEYGEN, [1])
    ct = c.encrypt(keys, np.arange(4.0), 3)
    r = c.rotate(keys, ct, 1)
    c.close()                 # the caller's reference ends; the handles still hold the context
    del keys, ct
    assert r.level == wl.L    # a handle still reads its own state
    del r                     # the last handle: the context goes with it


def test_layer_deeper_than_its_input(hk, tiny):
    """A layer evaluated on an input with too few levels stops with HE_EDEPTH
    (a clean error: no step goes below level 0)."""
    wl, layers, ctx, model, keys = tiny
    ct = ctx.encrypt(keys, synth.inputs(wl, 1, stream=5)[0], 11)
    for _ in range(wl.L - 2):
        ct = ctx.rescale(ct)
    assert ct.level == 2
    note("layer on a level-2 input")
    raises(hk, hk.HE_EDEPTH, ctx.eval_kan, model, keys, ct)
    # the context is usable afterwards and still exact
    top = ctx.encrypt(keys, synth.inputs(wl, 1, stream=5)[0], 11)
    r1 = ctx.eval_kan(model, keys, top).export()
    r2 = ctx.eval_kan(model, keys, top).export()
    assert (r1 == r2).all()
