"""The library's native continuous-batching server (he_server_create,
he_submit, he_poll) on the GPU: requests of two models submitted at once and
over time come back with exactly the residues of the same request evaluated
alone, requests submitted together share launches, a failing request reports
its error code, and tags that are not pending are refused."""
import sys
import time

import numpy as np
import pytest

from oracle import kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-server]", *a, flush=True)
    sys.stdout.flush()


def oracle_layers(name, ncal=512):
    wl = synth.WORKLOADS[name]
    raw = synth.raw_weights(wl)
    return kan.compile_model(raw, synth.calibration_inputs(wl, ncal), [wl.silu_degree] * len(raw),
                             [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)


@pytest.mark.timeout(900)
def test_native_server_results_equal_solo_results():
    from paper_2409_07751_amd import hekan
    wl = synth.WORKLOADS["image"]
    names = ["formula16", "tiny16"]
    layers = {n: oracle_layers(n) for n in names}
    ctx = hekan.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        models = {n: ctx.compile(layers[n]) for n in names}
        steps = sorted(set(s for m in models.values() for s in m.rotation_steps()))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        xs = {n: synth.inputs(synth.WORKLOADS[n], 8, stream=21) for n in names}
        reqs = []
        for i in range(12):
            n = names[i % 2]
            reqs.append((n, xs[n][i // 2], ctx.encrypt(keys, xs[n][i // 2], 400 + i)))
        # the solo results first: the server owns the context's stream while it exists
        solo = [ctx.eval_kan(models[n], keys, ct).export() for n, _, ct in reqs]
        ctx.sync()
        srv = hekan.NativeServer(ctx, keys, max_batch=8)
        try:
            note("submitting 8 at once, then 4 over time")
            tags = [srv.submit(models[n], ct) for n, _, ct in reqs[:8]]
            for n, _, ct in reqs[8:]:
                time.sleep(0.005)
                tags.append(srv.submit(models[n], ct))
            outs = []
            for t in tags:
                got = srv.poll(t, wait_ms=60000)
                assert got is not None
                outs.append(got)
            st = srv.stats()
            note(st)
            assert st["completed"] == 12 and st["layer_runs"] > st["layer_batches"]
            for (n, x, _), (ct, lat), want in zip(reqs, outs, solo):
                assert lat > 0
                assert (ct.export() == want).all(), "%s request differs from its solo run" % n
            # a tag already taken, and one never issued
            for bad in (tags[0], 10 ** 9):
                with pytest.raises(hekan.HeError) as e:
                    srv.poll(bad)
                assert e.value.code == hekan.HE_EINVAL
            # a request that cannot run (input at level 0): its error comes back through he_poll
            low = ctx.import_ct(np.zeros((2, 1, ctx.N), np.uint64), 0)
            t = srv.submit(models["tiny16"], low)
            with pytest.raises(hekan.HeError) as e:
                srv.poll(t, wait_ms=60000)
            assert e.value.code == hekan.HE_EDEPTH
            # a wrong number of input chunks is refused at submission
            with pytest.raises(hekan.HeError) as e:
                srv.submit(models["tiny16"], [reqs[0][2], reqs[0][2]])
            assert e.value.code == hekan.HE_ESHAPE
        finally:
            srv.close()
        y = ctx.decrypt(keys, outs[1][0], 1)
        assert np.abs(y - kan.he_friendly_kan(reqs[1][1][None], layers["tiny16"])[0]).max() < 1e-2
    finally:
        ctx.close()
