"""he_ct_rescale_noalloc (the rescale that allocates nothing) through the C
ABI: its output equals he_ct_rescale's residue for residue on two calls in a
row, the second with a smaller input, at N = 2^13 and at N = 2^16 with 25 Q
limbs; at N = 2^13 it also equals the oracle's rescale.  A rescale larger
than the library's scratch is refused with HE_ENOMEM and the context stays
usable; wrong output levels and an output that is the input are refused."""
import sys

import numpy as np
import pytest

from oracle import ckks as O
from paper_2409_07751_amd import synth

pytestmark = pytest.mark.gpu


def note(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hk():
    from paper_2409_07751_amd import hekan
    return hekan


def rand_res(ctx, q, level, seed):
    rng = np.random.default_rng(seed)
    return np.array([[rng.integers(0, int(q[l]), ctx.N, dtype=np.uint64) for l in range(level + 1)]
                     for _ in range(2)], np.uint64)


def check_two_calls(hk, ctx, levels, oracle_ctx=None):
    q, _, _ = ctx.primes()
    for i, lvl in enumerate(levels):
        note("N", ctx.N, "level", lvl)
        A = rand_res(ctx, q, lvl, 100 + lvl)
        a = ctx.import_ct(A, lvl)
        want = ctx.rescale(a).export()
        out = ctx.import_ct(rand_res(ctx, q, lvl - 1, 200 + lvl), lvl - 1)  # stale contents, overwritten
        got = ctx.rescale_noalloc(a, out).export()
        assert out.level == lvl - 1
        assert (got == want).all(), "call %d (level %d) differs from he_ct_rescale" % (i, lvl)
        if oracle_ctx is not None:
            o = O.Oracle(oracle_ctx).rescale(O.Ciphertext(lvl, A[0], A[1]))
            assert (got[0] == o.c0).all() and (got[1] == o.c1).all()


def test_noalloc_rescale_tiny(hk):
    wl = synth.WORKLOADS["tiny"]
    ctx = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        octx = O.Context(O.Params(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w))
        check_two_calls(hk, ctx, (wl.L, 3), octx)
        q, _, _ = ctx.primes()
        a = ctx.import_ct(rand_res(ctx, q, 3, 1), 3)
        with pytest.raises(hk.HeError) as e:  # output one level too high
            ctx.rescale_noalloc(a, ctx.import_ct(rand_res(ctx, q, 3, 2), 3))
        assert e.value.code == hk.HE_EINVAL
        # an output whose memory another ciphertext shares (a rotation by 0 returns its input)
        keys = ctx.keygen(synth.SEED_KEYGEN, [])
        o = ctx.import_ct(rand_res(ctx, q, 2, 4), 2)
        same = ctx.rotate(keys, o, 0)
        with pytest.raises(hk.HeError) as e:
            ctx.rescale_noalloc(a, same)
        assert e.value.code == hk.HE_EINVAL
        z = ctx.import_ct(rand_res(ctx, q, 0, 3), 0)
        with pytest.raises(hk.HeError) as e:  # nothing left to drop
            ctx.rescale_noalloc(z, z)
        assert e.value.code == hk.HE_EDEPTH
    finally:
        ctx.close()


def test_noalloc_rescale_image_top_level(hk):
    wl = synth.WORKLOADS["image"]
    ctx = hk.Context(wl.logN, wl.L, wl.scale_bits, wl.alpha, wl.w)
    try:
        check_two_calls(hk, ctx, (wl.L, 9))
    finally:
        ctx.close()


def test_noalloc_rescale_beyond_scratch_refused(hk):
    """N = 2^16 with 40 scale primes: a rescale of 41 limbs needs 41 MiB of
    staging, more than the 32 MiB the library holds."""
    ctx = hk.Context(16, 40, 45, 4, 5)
    try:
        q, _, _ = ctx.primes()
        a = ctx.import_ct(rand_res(ctx, q, 40, 5), 40)
        out = ctx.import_ct(rand_res(ctx, q, 39, 6), 39)
        with pytest.raises(hk.HeError) as e:
            ctx.rescale_noalloc(a, out)
        assert e.value.code == hk.HE_ENOMEM and "scratch" in str(e.value)
        # the context is still usable, and a rescale that fits runs
        check_two_calls(hk, ctx, (31, 12))
    finally:
        ctx.close()
