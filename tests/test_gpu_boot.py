"""CKKS bootstrapping on the GPU against the oracle's, bit for bit: key
material of the sparse secret, encryption at the top computation level,
ModRaise, multiplication by i, conjugation, CoeffToSlot, EvalMod,
SlotToCoeff and the whole refresh (single and batched) on the N = 2^11
bootstrappable parameter set; the refreshed ciphertext decrypts to its input
and computes.  All GPU work goes through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import boot as OB
from oracle import ckks as O
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-boot]", *a, flush=True)
    sys.stdout.flush()


def oparams(bs):
    return O.Params(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, bs.base_bits, bs.special_bits, bs.sigma,
                    bs.boot_levels, bs.boot_bits, bs.h)


def hctx(hk, bs):
    return hk.Context(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, base_bits=bs.base_bits,
                      special_bits=bs.special_bits, sigma=bs.sigma, boot_levels=bs.boot_levels,
                      boot_bits=bs.boot_bits, hamming_weight=bs.h)


def as_ct(c):
    return np.stack([c.c0, c.c1])


def imp(ctx, c):
    return ctx.import_ct(np.ascontiguousarray(as_ct(c)), c.level)


@pytest.fixture(scope="module")
def b11():
    from paper_2409_07751_amd import hekan
    bs = synth.BOOTSETS["boot11"]
    bp = OB.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)
    note("boot11 contexts")
    ctx = hctx(hekan, bs)
    octx = O.Context(oparams(bs))
    plan = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, bp.coeffs)
    steps = plan.rotation_steps()
    assert sorted(steps) == OB.rotation_steps(bs.logN, bp)
    keys = ctx.keygen(synth.SEED_KEYGEN, steps)
    okeys = O.Keys(octx, synth.SEED_KEYGEN, steps)
    ev = O.Oracle(octx, okeys)
    yield hekan, bs, bp, ctx, octx, plan, keys, ev
    del plan
    ctx.close()


def test_boot_chain_and_keys_equal_oracle(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    q, p, S = ctx.primes()
    assert (q == octx.q).all() and (p == octx.pm).all() and (S == octx.S).all()
    g = 2 * octx.p.N - 1
    assert g in keys.ek.ids()
    for kid in (0, g):
        for d in (0, 3):
            got = keys.ek.export(kid, d)
            assert (got == okeys_digit(ev, kid, d)).all(), (kid, d)


def okeys_digit(ev, kid, d):
    return ev.keys.keys[kid][d]


def test_encrypt_at_top_computation_level(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    z = synth.boot_inputs(bs, 1, stream=1)[0]
    ct = ctx.encrypt(keys, z, 77)
    assert ct.level == bs.Lc
    oc = ev.encrypt(z, 77)
    assert (ct.export() == as_ct(oc)).all()


def test_mod_raise_mul_i_conjugate_bit_exact(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    oc = ev.mod_drop(ev.encrypt(synth.boot_inputs(bs, 1, stream=2)[0], 78), 0)
    up = ctx.mod_raise(imp(ctx, oc))
    oup = ev.mod_raise(oc)
    assert up.level == bs.L and (up.export() == as_ct(oup)).all()
    assert (ctx.mul_i(up).export() == as_ct(ev.mul_i(oup))).all()
    low = ev.mod_drop(oup, 5)
    assert (ctx.rotate(keys, imp(ctx, low), hk.STEP_CONJUGATE).export() ==
            as_ct(ev.rotate(low, O.STEP_CONJUGATE))).all()
    assert (ctx.sub(imp(ctx, low), ctx.mul_i(imp(ctx, low))).export() == as_ct(ev.sub(low, ev.mul_i(low)))).all()


@pytest.fixture(scope="module")
def trace(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    oc = ev.mod_drop(ev.encrypt(synth.boot_inputs(bs, 1, stream=3)[0], 79), 1)
    tr = {}
    note("oracle bootstrap")
    out = OB.bootstrap(ev, oc, bp, tr)
    return oc, tr, out


def test_coeff_to_slot_bit_exact(b11, trace):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    oc, tr, _ = trace
    got = ctx.boot_coeff_to_slot(plan, keys, imp(ctx, oc))
    assert got.level == tr["cts"].level == bs.L - bs.cts
    assert (got.export() == as_ct(tr["cts"])).all()


def test_eval_mod_bit_exact(b11, trace):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    _, tr, _ = trace
    for y, u in zip(tr["split"], tr["evalmod"]):
        got = ctx.boot_eval_mod(plan, keys, imp(ctx, y))
        assert got.level == u.level
        assert (got.export() == as_ct(u)).all()


def test_slot_to_coeff_bit_exact(b11, trace):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    oc, tr, out = trace
    got = ctx.boot_slot_to_coeff(plan, keys, imp(ctx, tr["recombined"]), oc.level)
    assert got.level == out.level == bs.Lc
    assert (got.export() == as_ct(out)).all()


def test_bootstrap_bit_exact_and_accurate(b11, trace):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    oc, tr, out = trace
    got = ctx.bootstrap(plan, keys, imp(ctx, oc))
    assert got.level == bs.Lc
    assert (got.export() == as_ct(out)).all()
    want = ev.decrypt(oc, octx.p.slots)
    y = ctx.decrypt(keys, got, octx.p.slots)
    assert np.abs(y - want).max() < 1e-5
    # the refreshed ciphertext computes
    sq = ctx.mul(keys, got, got)
    assert np.abs(ctx.decrypt(keys, sq, octx.p.slots) - want * want).max() < 1e-5


def test_bootstrap_batch_equals_single(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    zs = synth.boot_inputs(bs, 3, stream=4)
    cts = [ctx.encrypt(keys, z, 90 + i) for i, z in enumerate(zs)]
    # one at level 0, as bootstrapping inputs usually arrive
    lows = [imp(ctx, ev.mod_drop(ev.encrypt(z, 90 + i), 0)) for i, z in enumerate(zs)]
    for group in (cts, lows):
        outs = ctx.bootstrap_batch(plan, keys, group)
        for c, o in zip(group, outs):
            assert (o.export() == ctx.bootstrap(plan, keys, c).export()).all()
    for z, o in zip(zs, ctx.bootstrap_batch(plan, keys, lows)):
        assert np.abs(ctx.decrypt(keys, o, len(z)) - z).max() < 1e-4


def test_bootstrap_errors(b11):
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    top = imp(ctx, ev.mod_raise(ev.mod_drop(ev.encrypt(np.zeros(4), 5), 0)))
    with pytest.raises(hk.HeError) as e:
        ctx.bootstrap(plan, keys, top)
    assert e.value.code == hk.HE_EINVAL
    nokeys = ctx.keygen(1, [1])
    with pytest.raises(hk.HeError) as e:
        ctx.bootstrap(plan, nokeys, ctx.encrypt(keys, np.zeros(4), 6))
    assert e.value.code == hk.HE_EKEY
    # a context without boot levels refuses a plan
    plain = hk.Context(bs.logN, bs.Lc, bs.scale_bits, bs.alpha, bs.w)
    try:
        with pytest.raises(hk.HeError) as e:
            plain.boot(bs.cts, bs.stc, bs.K, bs.r, bp.coeffs)
        assert e.value.code == hk.HE_EINVAL
    finally:
        plain.close()
    # a plan that needs more levels than the chain keeps
    deep = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, OB.cos_coeffs(bs.K, bs.r, 255))
    with pytest.raises(hk.HeError) as e:
        ctx.bootstrap(deep, keys, ctx.encrypt(keys, np.zeros(4), 7))
    assert e.value.code == hk.HE_EDEPTH


def kan_layers(name):
    from oracle import kan
    wl = synth.WORKLOADS[name]
    raw = synth.raw_weights(wl)
    return wl, kan.compile_model(raw, synth.calibration_inputs(wl, 512), [wl.silu_degree] * len(raw),
                                 [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)


@pytest.mark.parametrize("slots", [0, 64])
def test_kan_with_bootstrapping_between_layers_bit_exact(b11, slots):
    """The [2,5,1] KAN with a bootstrapping in place of the client-aided
    refresh: the whole inference on the server, residues equal to the
    oracle's, decrypted output within 1e-2 of the FP64 circuit; also with the
    sparse refresh of 64 slots (the layer output repeats with period 8)."""
    from oracle import circuit, kan
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    if slots:
        bp = OB.make_params(2, 2, bs.K, bs.r, bs.degree, slots=slots)
        plan = ctx.boot(2, 2, bs.K, bs.r, bp.coeffs, slots=slots)
    wl, layers = kan_layers("tiny16")
    model = ctx.compile(layers, refresh=True, circuit=hk.CIRCUIT_PAPER)
    steps = sorted(set(model.rotation_steps()) | set(plan.rotation_steps()))
    mkeys = ctx.keygen(synth.SEED_KEYGEN, steps)
    mev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
    x = synth.inputs(wl, 1)[0]
    ct = ctx.encrypt(mkeys, x, synth.SEED_ENC)
    note("oracle KAN with bootstrapping")
    want = circuit.eval_kan(mev, mev.encrypt(x, synth.SEED_ENC), layers,
                            refresh=lambda c, li: OB.bootstrap(mev, c, bp))
    got = ctx.eval_kan_boot(model, plan, mkeys, [ct])[0]
    assert got.level == want.level
    assert (got.export() == as_ct(want)).all()
    y = ctx.decrypt(mkeys, got, 1)
    assert abs(y[0] - kan.he_friendly_kan(x[None], layers)[0][0]) < 1e-2
    if slots:
        # the refreshed layer's output repeats with period 8: a plan of 4 slots is refused
        assert model.output_period(0) == 8
        small = ctx.boot(1, 1, bs.K, bs.r, bp.coeffs, slots=4)
        with pytest.raises(hk.HeError) as e:
            ctx.eval_kan_boot(model, small, mkeys, [ct])
        assert e.value.code == hk.HE_ESHAPE


def digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a.astype("<u8")).tobytes()).hexdigest()


@pytest.mark.timeout(900)
def test_boot16_full_size_equals_oracle_digests():
    """One bootstrapping at N = 2^16 (boot16) against the digests of the
    oracle's residues (tests/golden/boot_digests.json, written by
    make_boot_digests.py from the oracle alone): the encrypted input,
    CoeffToSlot and the refreshed output, bit for bit, then batched runs
    against the single one, and the decrypted error; the same for the
    real-slot refresh and for the sparsely packed refresh of 512 slots."""
    import json
    import os
    import time
    from paper_2409_07751_amd import hekan as hk
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "boot_digests.json")))
    bs = synth.BOOTSETS["boot16"]
    bp = OB.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)
    note("boot16 context")
    ctx = hctx(hk, bs)
    try:
        plan = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, bp.coeffs)
        steps = plan.rotation_steps()
        assert sorted(steps) == gold["steps"]
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        z = synth.boot_inputs(bs, 1)[0]
        ct = ctx.encrypt(keys, z, synth.SEED_ENC)
        st = gold["stages"]
        assert ct.level == st["input"]["level"] and digest(ct.export()) == st["input"]["sha256"]
        cts = ctx.boot_coeff_to_slot(plan, keys, ct)
        assert cts.level == st["cts"]["level"] and digest(cts.export()) == st["cts"]["sha256"]
        t = time.time()
        out = ctx.bootstrap(plan, keys, ct)
        ctx.sync()
        note("first bootstrap %.2f s (plaintexts encoded)" % (time.time() - t))
        e = out.export()
        for (p, l, n), v in zip(st["output"]["positions"], st["output"]["sampled"]):
            assert int(e[p][l][n]) == v, (p, l, n)
        assert out.level == st["output"]["level"] and digest(e) == st["output"]["sha256"]
        y = ctx.decrypt(keys, out, len(z))
        assert np.abs(y - z).max() < max(4 * gold["max_abs_err"], 1e-6)
        outs = ctx.bootstrap_batch(plan, keys, [ct, ct])
        assert all(digest(o.export()) == st["output"]["sha256"] for o in outs)
        del outs, out, cts, keys, plan
        # the real-slot refresh (SlotToCoeff first) of the same input
        rg = gold["real"]
        rbp = OB.make_params(bs.cts, bs.real_stc, bs.K, bs.r, bs.degree, real_slots=True)
        rplan = ctx.boot(bs.cts, bs.real_stc, bs.K, bs.r, rbp.coeffs, real_slots=True)
        assert sorted(rplan.rotation_steps()) == rg["steps"]
        rkeys = ctx.keygen(synth.SEED_KEYGEN, sorted(set(steps) | set(rg["steps"])))
        rct = ctx.encrypt(rkeys, z, synth.SEED_ENC)
        assert digest(rct.export()) == st["input"]["sha256"]
        rout = ctx.bootstrap(rplan, rkeys, rct)
        e = rout.export()
        for (p, l, n), v in zip(rg["stages"]["output"]["positions"], rg["stages"]["output"]["sampled"]):
            assert int(e[p][l][n]) == v, (p, l, n)
        assert rout.level == rg["stages"]["output"]["level"] and digest(e) == rg["stages"]["output"]["sha256"]
        y = ctx.decrypt(rkeys, rout, len(z))
        assert np.abs(y - z).max() < max(4 * rg["max_abs_err"], 1e-6)
        del rout, rct, rkeys, rplan
        # the sparsely packed refresh of 512 slots of a 512-periodic input
        sg = gold["sparse512"]
        sbp = OB.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree, slots=512)
        splan = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, sbp.coeffs, slots=512)
        assert sorted(splan.rotation_steps()) == sg["steps"]
        skeys = ctx.keygen(synth.SEED_KEYGEN, sg["steps"])
        zs = np.tile(z[:512], len(z) // 512)
        sct = ctx.encrypt(skeys, zs, synth.SEED_ENC)
        ss = sg["stages"]
        assert digest(sct.export()) == ss["input"]["sha256"]
        scts = ctx.boot_coeff_to_slot(splan, skeys, sct)
        assert scts.level == ss["cts"]["level"] and digest(scts.export()) == ss["cts"]["sha256"]
        sout = ctx.bootstrap(splan, skeys, sct)
        e = sout.export()
        for (p, l, n), v in zip(ss["output"]["positions"], ss["output"]["sampled"]):
            assert int(e[p][l][n]) == v, (p, l, n)
        assert sout.level == ss["output"]["level"] and digest(e) == ss["output"]["sha256"]
        y = ctx.decrypt(skeys, sout, len(zs))
        assert np.abs(y - zs).max() < max(4 * sg["max_abs_err"], 1e-6)
    finally:
        ctx.close()


def test_deep_comparison_kan_with_bootstrapping_reaches_the_exact_kan():
    """What bootstrapping buys: the tiny KAN with a depth-12 comparison
    composite (17 levels per layer, more than any client-refresh budget here)
    runs whole on the server with a refresh between layers (boot11deep); the
    first request's residues equal the oracle's, and every request decrypts
    within 1e-4 of its FP64 circuit and within 1e-2 of the exact KAN."""
    from oracle import circuit, kan
    from paper_2409_07751_amd import hekan as hk
    bs = synth.BOOTSETS["boot11deep"]
    bp = OB.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)
    wl, layers = kan_layers("tinydeep")
    ctx = hctx(hk, bs)
    octx = O.Context(oparams(bs))
    try:
        plan = ctx.boot(bs.cts, bs.stc, bs.K, bs.r, bp.coeffs)
        model = ctx.compile(layers, refresh=True, circuit=hk.CIRCUIT_PAPER)
        steps = sorted(set(model.rotation_steps()) | set(plan.rotation_steps()))
        keys = ctx.keygen(synth.SEED_KEYGEN, steps)
        ev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
        xs = synth.inputs(wl, 4, stream=5)
        cts = [ctx.encrypt(keys, x, synth.SEED_ENC + i) for i, x in enumerate(xs)]
        outs = ctx.eval_kan_boot(model, plan, keys, cts)
        note("oracle deep KAN with bootstrapping")
        want = circuit.eval_kan(ev, ev.encrypt(xs[0], synth.SEED_ENC), layers,
                                refresh=lambda c, li: OB.bootstrap(ev, c, bp))
        assert outs[0].level == want.level and (outs[0].export() == as_ct(want)).all()
        o2 = kan.he_friendly_kan(xs, layers)[:, 0]
        o3 = kan.exact_kan(xs, layers)[:, 0]
        y = np.array([ctx.decrypt(keys, o, 1)[0] for o in outs])
        note("|y - O2| %.3g, |y - O3| %.3g" % (np.abs(y - o2).max(), np.abs(y - o3).max()))
        assert np.abs(y - o2).max() < 1e-4 and np.abs(y - o3).max() < 1e-2
        del outs, cts, keys, model, plan
    finally:
        ctx.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("real,slots", [(False, 0), (True, 0), (True, 512)])
def test_formula_kan_with_bootstrapping_at_n16(real, slots):
    """The [4,10,10,1] formula KAN (restructured, three 8-level layers) at
    N = 2^16 with a refresh between layers (boot16, the full-slot refresh,
    the real-slot one with SlotToCoeff first, or that one sparsely packed on
    512 slots, the layer outputs repeating with period 16): four requests in one batch
    decrypt within 1e-2 of the FP64 circuit, and the batch equals the
    requests run one at a time, bit for bit."""
    from oracle import kan
    from paper_2409_07751_amd import hekan as hk
    bs = synth.BOOTSETS["boot16"]
    bp = OB.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)
    wl, layers = kan_layers("formula16")
    ctx = hctx(hk, bs)
    try:
        plan = ctx.boot(bs.cts, bs.real_stc if real else bs.stc, bs.K, bs.r, bp.coeffs, real_slots=real, slots=slots)
        model = ctx.compile(layers, refresh=True, circuit=hk.CIRCUIT_RESTRUCTURED)
        keys = ctx.keygen(synth.SEED_KEYGEN, sorted(set(model.rotation_steps()) | set(plan.rotation_steps())))
        xs = synth.inputs(wl, 4, stream=6)
        cts = [ctx.encrypt(keys, x, synth.SEED_ENC + i) for i, x in enumerate(xs)]
        outs = ctx.eval_kan_boot(model, plan, keys, cts)
        y = np.array([ctx.decrypt(keys, o, 1)[0] for o in outs])
        want = kan.he_friendly_kan(xs, layers)[:, 0]
        note("formula16 with bootstrapping: max |y - FP64 circuit| %.3g" % np.abs(y - want).max())
        assert np.abs(y - want).max() < 1e-2
        for c, o in zip(cts[:2], outs[:2]):
            assert (ctx.eval_kan_boot(model, plan, keys, [c])[0].export() == o.export()).all()
        del outs, cts, keys, model, plan
    finally:
        ctx.close()



def test_real_slot_refresh_bit_exact(b11):
    """The real-slot refresh with SlotToCoeff first (he_boot_desc.real_slots)
    against the oracle's, bit for bit, from the lowest level it accepts and
    from the top computation level; batches equal single refreshes; an input
    below stc_levels is refused."""
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    rbp = OB.make_params(bs.cts, bs.real_stc, bs.K, bs.r, bs.degree, real_slots=True)
    rplan = ctx.boot(bs.cts, bs.real_stc, bs.K, bs.r, rbp.coeffs, real_slots=True)
    assert set(rplan.rotation_steps()) <= set(plan.rotation_steps())  # the keys b11 made
    zs = synth.boot_inputs(bs, 3, stream=8)
    for lvl in (bs.real_stc, bs.Lc):
        ocs = [ev.mod_drop(ev.encrypt(z, 120 + i), lvl) for i, z in enumerate(zs)]
        want = [OB.bootstrap(ev, oc, rbp) for oc in ocs]
        got = ctx.bootstrap(rplan, keys, imp(ctx, ocs[0]))
        assert got.level == bs.Lc and (got.export() == as_ct(want[0])).all()
        outs = ctx.bootstrap_batch(rplan, keys, [imp(ctx, oc) for oc in ocs])
        for o, w, oc in zip(outs, want, ocs):
            assert (o.export() == as_ct(w)).all()
            assert np.abs(ctx.decrypt(keys, o, octx.p.slots) - ev.decrypt(oc, octx.p.slots)).max() < 1e-6
    with pytest.raises(hk.HeError) as e:
        ctx.bootstrap(rplan, keys, imp(ctx, ev.mod_drop(ev.encrypt(zs[0], 5), bs.real_stc - 1)))
    assert e.value.code == hk.HE_EINVAL
    # he_ct_mod_drop gives the oracle's mod-drop
    low = ctx.mod_drop(ctx.encrypt(keys, zs[1], 121), bs.real_stc)
    assert low.level == bs.real_stc and (low.export() == as_ct(ev.mod_drop(ev.encrypt(zs[1], 121), bs.real_stc))).all()
    with pytest.raises(hk.HeError) as e:
        ctx.mod_drop(low, bs.real_stc + 1)
    assert e.value.code == hk.HE_EINVAL


@pytest.mark.parametrize("n,real", [(8, False), (64, False), (256, False), (64, True), (256, True)])
def test_sparse_refresh_bit_exact(b11, n, real):
    """The sparsely packed refresh (he_boot_desc.slots = n: SubSum, then the
    transforms' first log2 n stages; with real_slots, SlotToCoeff first) of
    n-periodic messages against the oracle's, bit for bit, single and batched,
    and within 1e-6 of the input; slots that are not a power of two or above
    N/2, or more stage groups than log2 n, are refused."""
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    G = 1 if n == 8 else 2
    sbp = OB.make_params(G, G, bs.K, bs.r, bs.degree, real_slots=real, slots=n)
    splan = ctx.boot(G, G, bs.K, bs.r, sbp.coeffs, real_slots=real, slots=n)
    steps = splan.rotation_steps()
    assert sorted(steps) == OB.rotation_steps(bs.logN, sbp)
    note("sparse refresh, slots", n, "keys", len(steps))
    skeys = ctx.keygen(synth.SEED_KEYGEN, steps)
    sev = O.Oracle(octx, O.Keys(octx, synth.SEED_KEYGEN, steps))
    M = octx.p.slots
    zs = [np.tile(np.random.default_rng(n + i).uniform(-1, 1, n), M // n) for i in range(2)]
    ocs = [sev.mod_drop(sev.encrypt(z, 140 + i), G if real else 1) for i, z in enumerate(zs)]
    want = [OB.bootstrap(sev, oc, sbp) for oc in ocs]
    got = ctx.bootstrap(splan, skeys, imp(ctx, ocs[0]))
    assert got.level == bs.Lc and (got.export() == as_ct(want[0])).all()
    outs = ctx.bootstrap_batch(splan, skeys, [imp(ctx, oc) for oc in ocs])
    for o, w, z in zip(outs, want, zs):
        assert (o.export() == as_ct(w)).all()
        assert np.abs(ctx.decrypt(keys, o, M) - z).max() < 1e-6
    for args, kw in (((1, 1), {"slots": n + 1}), ((1, 1), {"slots": 2 * M}), ((G + 8, 1), {"slots": n}),
                     ((1, G + 8), {"real_slots": True, "slots": n})):
        with pytest.raises(hk.HeError) as e:
            ctx.boot(*args, bs.K, bs.r, sbp.coeffs, **kw)
        assert e.value.code == hk.HE_EINVAL


@pytest.mark.parametrize("real,n,slots", [(False, 2, 0), (True, 1, 0), (True, 2, 64)])
def test_graph_bootstrap_replays_equal_eager(b11, real, n, slots):
    """A refresh captured into a HIP graph (he_graph_capture_bootstrap): every
    replay, with eager work of the same context between replays, reproduces
    the eager result bit for bit (full-slot, real-slot and sparse real-slot
    plans)."""
    hk, bs, bp, ctx, octx, plan, keys, ev = b11
    stc = bs.real_stc if real else bs.stc
    pl = ctx.boot(bs.cts, stc, bs.K, bs.r, bp.coeffs, real_slots=real, slots=slots) if real else plan
    if slots:
        keys = ctx.keygen(synth.SEED_KEYGEN, pl.rotation_steps())
    zs = synth.boot_inputs(bs, n, stream=9)
    if slots:
        zs = [np.tile(z[:slots], len(z) // slots) for z in zs]
    ocs = [ev.mod_drop(ev.encrypt(z, 140 + i), 3) for i, z in enumerate(zs)]
    cts = [imp(ctx, oc) for oc in ocs[:n]]
    eager = [o.export() for o in ctx.bootstrap_batch(pl, keys, cts)]
    note("capture bootstrap, real", real, "batch", n)
    graph, outs = ctx.graph_capture_bootstrap(pl, keys, cts)
    ctx.sync()
    for i in range(n):
        assert (outs[i].export() == eager[i]).all(), "captured run, input %d" % i
    for rep in range(3):
        other = ctx.bootstrap_batch(pl, keys, cts[::-1])
        graph.launch()
        ctx.sync()
        for i in range(n):
            assert (outs[i].export() == eager[i]).all(), "replay %d, input %d" % (rep, i)
            assert (other[n - 1 - i].export() == eager[i]).all(), "eager run between replays"
    graph.free()
    assert (outs[0].export() == eager[0]).all()
