"""The client/server key split of the C ABI (the paper's threat model: the
client keeps the secret key, the server evaluates with evaluation keys
alone).  A server context that never sees a secret key builds its
evaluation keys from the material the client exports, evaluates a KAN layer
on the client's ciphertext (moved between contexts as residues), and its
result equals the client-side evaluation residue for residue; the client
decrypts it within 1e-2 of the FP64 circuit.  Import refuses malformed key
material, and a product without a relinearisation key reports HE_EKEY."""
import sys

import numpy as np
import pytest

from oracle import ckks as O
from oracle import kan
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-keys]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hk():
    from paper_2409_07751_amd import hekan
    return hekan


def test_server_evaluates_with_imported_keys_only(hk):
    wl = synth.WORKLOADS["tiny"]
    layers = kan.compile_model(synth.raw_weights(wl), synth.calibration_inputs(wl), [wl.silu_degree] * 2,
                               [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    client = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    server = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        cmodel = client.compile(layers[:1])
        steps = cmodel.rotation_steps()
        keys = client.keygen(synth.SEED_KEYGEN, steps)
        octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
        galois = sorted(octx.galois_elt(s) for s in steps)
        assert keys.ek.ids() == [0] + galois
        note("export", len(galois) + 1, "keys")
        material = keys.ek.export_all()
        server_ek = server.import_eval_keys(material)
        assert server_ek.ids() == keys.ek.ids()
        for i in (0, galois[0], galois[-1]):  # the imported keys export the same residues
            assert (server_ek.export(i, 3) == material[i][3]).all()
        x = synth.inputs(wl, 1)[0]
        ct = client.encrypt(keys, x, synth.SEED_ENC)
        want = client.eval_kan(cmodel, keys, ct)
        note("server evaluation")
        smodel = server.compile(layers[:1])
        sct = server.import_ct(ct.export(), ct.level)
        out = server.eval_kan(smodel, server_ek, sct)
        got = out.export()
        assert (got == want.export()).all()
        back = client.import_ct(got, out.level)
        y = client.decrypt(keys, back, layers[0].n_out)
        assert np.abs(y - kan.he_friendly_layer(x[None], layers[0])[0]).max() < 1e-2
        # the server holds evaluation keys only: a secret-key call cannot take them
        with pytest.raises(TypeError):
            server.encrypt(server_ek, x, 1)
    finally:
        client.close()
        server.close()


def test_import_refuses_bad_material(hk):
    wl = synth.WORKLOADS["tiny"]
    ctx = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        keys = ctx.keygen(synth.SEED_KEYGEN, [1])
        m = keys.ek.export_all()
        g = [i for i in m if i][0]

        def refused(material, code):
            with pytest.raises(hk.HeError) as e:
                ctx.import_eval_keys(material)
            assert e.value.code == code, str(e.value)

        refused({2: m[g]}, hk.HE_EINVAL)                       # 2 is not a Galois element
        bad = m[0].copy()
        bad[0, 0, 0, 0] = np.uint64(2) ** np.uint64(62)          # unreduced residue
        refused({0: bad}, hk.HE_EINVAL)
        # Galois keys alone: rotations work, a product has no relinearisation key
        only = ctx.import_eval_keys({g: m[g]})
        ct = ctx.encrypt(keys, np.arange(8.0) / 8, 2)
        assert (ctx.rotate(only, ct, 1).export() == ctx.rotate(keys, ct, 1).export()).all()
        with pytest.raises(hk.HeError) as e:
            ctx.mul(only, ct, ct)
        assert e.value.code == hk.HE_EKEY
    finally:
        ctx.close()
