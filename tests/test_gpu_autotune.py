"""Key-switch configurations (he_ctx_set_keyswitch / he_ctx_autotune): every
configuration at every level gives the residues of the default one, and the
autotuner's choices are valid configurations."""
import sys

import pytest

from oracle import kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu

CONFIGS = (0, 1, 8, 32)


def note(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def setup(hekan, name, nlayers):
    wl = synth.WORKLOADS[name]
    raw = synth.raw_weights(wl)
    layers = kan.compile_model(raw, synth.calibration_inputs(wl, 1024), [wl.silu_degree] * 2,
                               [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    ctx = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    model = ctx.compile(layers[:nlayers])
    keys = ctx.keygen(synth.SEED_KEYGEN, model.rotation_steps())
    return wl, ctx, model, keys


@pytest.mark.parametrize("name,nlayers,nb", [("tiny", 1, 3), ("image", 2, 2)])
def test_every_configuration_same_residues(name, nlayers, nb):
    from paper_2409_07751_amd import hekan
    note("context", name)
    wl, ctx, model, keys = setup(hekan, name, nlayers)
    try:
        xs = synth.inputs(wl, nb, stream=17)
        cts = [ctx.encrypt(keys, xs[i], 90 + i) for i in range(nb)]
        ref = [o.export() for o in ctx.eval_kan_batch(model, keys, cts)]
        for cfg in CONFIGS:
            for lvl in range(wl.L + 1):
                ctx.set_keyswitch(lvl, nb, cfg)
            note(name, "configuration", cfg)
            outs = ctx.eval_kan_batch(model, keys, cts)
            for i in range(nb):
                assert (outs[i].export() == ref[i]).all(), "configuration %d, request %d" % (cfg, i)
        choice = ctx.autotune(keys, nb, reps=2)
        note(name, "autotuned", choice)
        assert len(choice) == wl.L + 1 and all(c in CONFIGS for c in choice)
        assert choice[0] == 0  # no FP64 limb to fuse at level 0
        outs = ctx.eval_kan_batch(model, keys, cts)
        for i in range(nb):
            assert (outs[i].export() == ref[i]).all(), "autotuned, request %d" % i
        with pytest.raises(hekan.HeError) as e:
            ctx.set_keyswitch(0, nb, 5)
        assert e.value.code == hekan.HE_EINVAL
        with pytest.raises(hekan.HeError) as e:
            ctx.set_keyswitch(wl.L + 1, nb, 8)
        assert e.value.code == hekan.HE_EINVAL
    finally:
        ctx.close()
