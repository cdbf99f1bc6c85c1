"""Pins of the oracle's CKKS bootstrapping against mathematics that does not
depend on it: the special DFT of the encoding written out from its definition
(zeta^(5^j k)), big-integer reconstruction of the ModRaise plaintext, the
closed form sin(2 pi y), conjugation and multiplication by i on decrypted
slots, and the refreshed ciphertext decrypting to its input."""
import math

import numpy as np
import pytest

from oracle import boot, ckks
from oracle.ckks import P, Params, lib
from paper_2409_07751_amd import synth


def bootset_params(bs):
    return Params(bs.logN, bs.L, bs.scale_bits, bs.alpha, bs.w, bs.base_bits, bs.special_bits, bs.sigma,
                  bs.boot_levels, bs.boot_bits, bs.h)


def bootset_bp(bs):
    return boot.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree)


def special_dft(logN):
    N = 1 << logN
    M = N // 2
    e = np.array([[pow(5, j, 2 * N) * k % (2 * N) for k in range(M)] for j in range(M)])
    return np.exp(1j * np.pi * e / N)


def bit_reversal(m):
    M = 1 << m
    R = np.zeros((M, M))
    for i in range(M):
        R[i, int(format(i, "0%db" % m)[::-1], 2) if m else 0] = 1
    return R


def dense(logN, stages, inverse):
    M = 1 << (logN - 1)
    I, J, S, E = boot.group_terms(logN, stages, inverse)
    A = np.zeros((M, M), complex)
    A[I, J] = S * (0.5 ** len(stages) if inverse else 1.0) * np.exp(1j * np.pi * E / (1 << logN))
    return A


@pytest.mark.parametrize("logN", [3, 5, 7, 8])
def test_butterfly_stages_factor_the_special_dft(logN):
    """F_{m-1} ... F_0 R = U0 and (F_0^H/2) ... (F_{m-1}^H/2) = (2/N) R U0^H,
    for every grouping of the stages."""
    N, m = 1 << logN, logN - 1
    U0, R = special_dft(logN), bit_reversal(m)
    for G in range(1, m + 1):
        A = np.eye(1 << m)
        for st in boot.stage_groups(m, G, True):
            A = dense(logN, st, False) @ A
        assert np.abs(A @ R - U0).max() < 1e-12
        B = np.eye(1 << m)
        for st in boot.stage_groups(m, G, False):
            B = dense(logN, st, True) @ B
        assert np.abs(B - (2.0 / N) * R @ U0.conj().T).max() < 1e-13


@pytest.mark.parametrize("logN,n", [(6, 2), (6, 8), (7, 16), (8, 32)])
def test_first_stages_are_the_sparse_special_dft_on_every_block(logN, n):
    """The sparse packing's transform: F_{log2 n - 1} ... F_0 of the full
    factorisation is block diagonal, every aligned block of n being the n-slot
    special DFT U0'[j][k] = zeta'^(5^j k) (zeta' = exp(i pi / (2 n)), a
    primitive 4n-th root) times the n-point bit reversal; and its inverse
    stages (F^H/2) give (1/n) R' U0'^H on every block."""
    M, m = 1 << (logN - 1), n.bit_length() - 1
    e = np.array([[pow(5, j, 4 * n) * k % (4 * n) for k in range(n)] for j in range(n)])
    U = np.exp(1j * np.pi * e / (2 * n))
    R = bit_reversal(m)
    A = np.eye(M)
    for st in boot.stage_groups(m, min(2, m), True):
        A = dense(logN, st, False) @ A
    B = np.eye(M)
    for st in boot.stage_groups(m, min(2, m), False):
        B = dense(logN, st, True) @ B
    for b in range(M // n):
        blk = slice(b * n, (b + 1) * n)
        assert np.abs(A[blk, blk] @ R - U).max() < 1e-12
        assert np.abs(B[blk, blk] - R @ U.conj().T / n).max() < 1e-13
        A[blk, blk] = 0
        B[blk, blk] = 0
    assert np.abs(A).max() == 0 and np.abs(B).max() == 0


def test_group_diagonals_are_the_group_matrix():
    logN = 7
    M = 1 << (logN - 1)
    st = [4, 3, 2]
    A = dense(logN, st, True) * 0.3
    D = boot.group_diagonals(logN, st, True, 0.3)
    assert len(D) == 2 ** (len(st) + 1) - 1
    B = np.zeros((M, M), complex)
    for o, (re, im) in D.items():
        for i in range(M):
            B[i, (i + o) % M] += re[i] + 1j * im[i]
    assert np.abs(A - B).max() < 1e-15
    # the top group's offsets wrap around: M/u distinct rotations
    Dt = boot.group_diagonals(logN, [5, 4], True, 1.0)
    assert sorted(Dt) == [-16, 0, 16, 32]


def dec_cos_sin(num, den):
    """cos and sin of pi num / den to 50 digits (decimal Taylor series; pi by
    Machin's formula)"""
    from decimal import Decimal, getcontext
    getcontext().prec = 60

    def arctan_inv(x):
        x = Decimal(x)
        t, s, k = 1 / x, 1 / x, 1
        while abs(t) > Decimal(10) ** -58:
            t = -t / (x * x)
            s += t / (2 * k + 1)
            k += 1
        return s

    pi = 16 * arctan_inv(5) - 4 * arctan_inv(239)
    a = pi * num / den
    c, s, t, k = Decimal(0), Decimal(0), Decimal(1), 0
    while abs(t) > Decimal(10) ** -58 or k < 4:
        if k % 2 == 0:
            c += t if k % 4 == 0 else -t
        else:
            s += t if k % 4 == 1 else -t
        k += 1
        t = t * a / k
    return c, s


def test_root_table_is_nearest_double():
    logN = 6
    N = 1 << logN
    re, im = boot.root_table(logN)
    exact = {0: (1.0, 0.0), N // 2: (0.0, 1.0), N: (-1.0, 0.0), 3 * N // 2: (0.0, -1.0)}
    for e in range(2 * N):
        c, s = exact.get(e) or [float(v) for v in dec_cos_sin(e, N)]
        assert re[e] == c and im[e] == s, e


def test_cosine_series_and_evalmod_closed_form():
    for K, r, deg in [(12.0, 4, 23), (32.0, 5, 31)]:
        bp = boot.make_params(2, 2, K, r, deg)
        # the interpolant equals the function at its Chebyshev nodes
        n = deg + 1
        u = np.cos(np.pi * (np.arange(n) + 0.5) / n)
        f = np.cos(2 * np.pi * (K * u - 0.25) / 2 ** r)
        assert np.abs(np.polynomial.chebyshev.chebval(u, bp.coeffs) - f).max() < 1e-13
        # EvalMod = sin(2 pi y) near every integer of the range
        y = (np.arange(-K + 1, K)[:, None] + np.linspace(-1e-3, 1e-3, 21)[None, :]).ravel()
        assert np.abs(boot.evalmod_plain(y, bp) - np.sin(2 * np.pi * y)).max() < 1e-11


@pytest.mark.parametrize("name", sorted(synth.BOOTSETS))
def test_boot_level_plan_fits_the_boot_levels(name):
    """CoeffToSlot, EvalMod and SlotToCoeff of each bootstrappable parameter set
    use exactly its boot levels (levels traced on the slot simulator)."""
    from oracle.slotsim import SlotSim
    bs = synth.BOOTSETS[name]
    bp = bootset_bp(bs)
    sim = SlotSim(16)
    y = sim.fresh(np.linspace(-bs.K + 0.5, bs.K - 0.5, 16), bs.L - bs.cts)
    u = boot.eval_mod(sim, y, bp)
    assert np.abs(u.v - np.sin(2 * np.pi * y.v)).max() < 1e-10
    assert bs.cts + (bs.L - bs.cts - u.level) + bs.stc == bs.boot_levels


def test_sparse_ternary_secret():
    L = lib()
    s = np.zeros(1 << 11, np.int64)
    L.oc_sample_sparse_ternary(5, 1, 0, 0, 11, 32, P(s))
    assert (s != 0).sum() == 32 and set(np.unique(s)) <= {-1, 0, 1}
    s2 = np.zeros(1 << 11, np.int64)
    L.oc_sample_sparse_ternary(5, 1, 0, 0, 11, 32, P(s2))
    assert (s == s2).all()
    L.oc_sample_sparse_ternary(6, 1, 0, 0, 11, 32, P(s2))
    assert (s != s2).any()
    big = np.zeros(1 << 16, np.int64)
    L.oc_sample_sparse_ternary(5, 1, 0, 0, 16, 20000, P(big))
    assert (big != 0).sum() == 20000 and abs((big == 1).mean() - (big == -1).mean()) < 0.01
    # positions spread over the whole ring
    assert abs(np.flatnonzero(big).mean() / (1 << 16) - 0.5) < 0.01
    L.oc_sample_sparse_ternary(5, 1, 0, 0, 4, 16, P(big))
    assert (big[:16] != 0).all()


def test_boot_chain():
    bs = synth.BOOTSETS["boot16"]
    p = bootset_params(bs)
    ctx = ckks.Context(p)
    M2 = 2 << bs.logN
    allp = [int(v) for v in list(ctx.q) + list(ctx.pm)]
    assert len(set(allp)) == len(allp) and all(v % M2 == 1 for v in allp)
    top = p.top_level
    assert top == bs.Lc and ctx.S[bs.L] == 2.0 ** bs.boot_bits and ctx.S[top] == 2.0 ** bs.scale_bits
    for l in range(bs.L, 0, -1):
        bits = bs.boot_bits if l > top else bs.scale_bits
        assert abs(math.log2(int(ctx.q[l])) - bits) < 0.01
        if l != top + 1:
            assert ctx.S[l - 1] == ctx.S[l] * ctx.S[l] / float(ctx.q[l])
    # without boot levels the chain is the computation chain alone
    plain = ckks.Context(Params(bs.logN, bs.Lc, bs.scale_bits, bs.alpha, bs.w, bs.base_bits))
    assert [int(v) for v in plain.q] == [int(v) for v in ctx.q[:1]] + [int(v) for v in plain.q[1:]]


@pytest.fixture(scope="module")
def boot11():
    bs = synth.BOOTSETS["boot11"]
    p = bootset_params(bs)
    ctx = ckks.Context(p)
    bp = bootset_bp(bs)
    keys = ckks.Keys(ctx, synth.SEED_KEYGEN, boot.rotation_steps(bs.logN, bp) + [1])
    return bs, p, ctx, bp, keys, ckks.Oracle(ctx, keys)


def test_conjugation_and_mul_i(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, p.slots) + 1j * rng.uniform(-1, 1, p.slots)
    l = p.top_level
    m = ev.encode(z, ctx.S[l], l + 1)
    ct = ev.encrypt(np.zeros(4), 9)
    ct = ckks.Ciphertext(l, ev._binop(ev.lib.oc_poly_add, ct.c0, m, l + 1), ct.c1)
    assert np.abs(ev.decrypt_c(ct, p.slots) - z).max() < 1e-6
    assert np.abs(ev.decrypt_c(ev.rotate(ct, ckks.STEP_CONJUGATE), p.slots) - np.conj(z)).max() < 1e-6
    assert np.abs(ev.decrypt_c(ev.mul_i(ct), p.slots) - 1j * z).max() < 1e-6
    assert np.abs(ev.decrypt_c(ev.rotate(ct, 1), p.slots) - np.roll(z, -1)).max() < 1e-6


def test_complex_encoder_matches_direct_sum(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    L = lib()
    rng = np.random.default_rng(4)
    re, im = rng.uniform(-2, 2, 300), rng.uniform(-2, 2, 300)
    scale = 2.0 ** 40 * 1.37
    m = ev.encode(re + 1j * im, scale, 1)
    q0 = int(ctx.q[0])
    for i in (0, 3, 700, 1024, 2047):
        d = L.oc_encode_coeff_direct_c(P(re), P(im), 300, scale, bs.logN, i)
        v = int(m[0, i])
        v = v - q0 if v > q0 // 2 else v
        assert abs(v - d) <= 0.5 + 1e-9 * scale
    # real slots through the complex path give the real encoder's residues
    mr = ev.encode(re, scale, 2)
    mc = ev.encode(re + 0j, scale, 2)
    assert (mr == mc).all()


def test_mod_raise_adds_a_multiple_of_q0(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    ct = ev.mod_drop(ev.encrypt(synth.boot_inputs(bs, 1)[0], 21), 0)
    up = ev.mod_raise(ct)
    assert up.level == p.L
    q = [int(v) for v in ctx.q]
    s = keys.s_small
    N = p.N

    def phase_int(c, mods):
        # c0 + c1 s over the integers from the residues (CRT over `mods` limbs), centred
        res = []
        for t in range(len(mods)):
            a = np.zeros((1, N), np.uint64)
            lib().oc_poly_mul(P(np.ascontiguousarray(c.c1[t:t + 1])),
                              P(np.ascontiguousarray(keys.s_res[t:t + 1])), P(a), 1, p.logN,
                              P(ckks.u64a([mods[t]])))
            res.append([(int(x) + int(y)) % mods[t] for x, y in zip(a[0], c.c0[t])])
        Q = math.prod(mods)
        out = []
        for k in range(N):
            x = sum(r[k] * (Q // mm) * pow(Q // mm, -1, mm) for r, mm in zip(res, mods)) % Q
            out.append(x - Q if x > Q // 2 else x)
        return np.array(out, dtype=object)

    t_small = phase_int(ct, q[:1])
    t_big = phase_int(up, q[:3])
    I = (t_big - t_small) // q[0]
    assert all((tb - ts) % q[0] == 0 for tb, ts in zip(t_big, t_small))
    assert max(abs(int(v)) for v in I) <= (bs.h + 1) // 2
    assert max(abs(int(v)) for v in I) <= bs.K


def decrypt_wide(ev, ct, nlimbs=2):
    """complex slots of a ciphertext whose message exceeds q_0 / 2: the phase
    reconstructed over the first nlimbs limbs (CRT), centred, then decoded"""
    ctx, p = ev.ctx, ev.ctx.p
    mods = [int(v) for v in ctx.q[:nlimbs]]
    res = []
    for t in range(nlimbs):
        a = np.zeros((1, p.N), np.uint64)
        m = ckks.u64a([mods[t]])
        lib().oc_poly_mul(P(np.ascontiguousarray(ct.c1[t:t + 1])), P(np.ascontiguousarray(ev.keys.s_res[t:t + 1])),
                          P(a), 1, p.logN, P(m))
        lib().oc_poly_add(P(a), P(np.ascontiguousarray(ct.c0[t:t + 1])), P(a), 1, p.logN, P(m))
        res.append(a[0])
    Q = math.prod(mods)
    big = []
    for k in range(p.N):
        x = sum(int(r[k]) * (Q // mm) * pow(Q // mm, -1, mm) for r, mm in zip(res, mods)) % Q
        x = x - Q if x > Q // 2 else x
        assert abs(x) < 2 ** 62
        big.append(x % 2 ** 63)
    return _decode63(ev, big, ct)


def _decode63(ev, big, ct):
    p = ev.ctx.p
    re = np.zeros(p.slots)
    im = np.zeros(p.slots)
    lib().oc_decode_c(P(np.array(big, np.uint64)), 2 ** 63, ev.ctx.S[ct.level], p.logN, p.slots, P(re), P(im))
    return re + 1j * im


def test_bootstrap_refreshes_to_the_top_computation_level(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    z = synth.boot_inputs(bs, 1)[0]
    ct = ev.mod_drop(ev.encrypt(z, 22), 1)
    want = ev.decrypt(ct, p.slots)
    tr = {}
    out = boot.bootstrap(ev, ct, bp, tr)
    assert out.level == p.top_level
    assert tr["cts"].level == p.L - bs.cts
    got = ev.decrypt_c(out, p.slots)
    assert np.abs(got.real - want).max() < 1e-5
    assert np.abs(got.imag).max() < 1e-5
    # the refreshed ciphertext computes: its square at the next level
    sq = ev.mul(out, out)
    assert np.abs(ev.decrypt(sq, p.slots) - want * want).max() < 1e-5
    # CoeffToSlot puts (t_k + i t_{k+N/2}) / (2 q0) in bit-reversed slot k: its
    # real parts near integers plus m_k / (2 q0), all within [-K/2, K/2]
    w = decrypt_wide(ev, tr["cts"])
    assert np.abs(w.real).max() <= bs.K / 2 and np.abs(w.imag).max() <= bs.K / 2
    frac = 2 * w.real - np.round(2 * w.real)
    assert np.abs(frac).max() < 1e-3


def test_bootstrap_rotation_steps_cover_its_rotations(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    steps = boot.rotation_steps(bs.logN, bp)
    assert ckks.STEP_CONJUGATE in steps
    used = []

    class Spy(ckks.Oracle):
        def rotate(self, a, t):
            used.append(t)
            return super().rotate(a, t)

        def rotate_sum(self, items):
            used.extend(t for _, t in items if t)
            return super().rotate_sum(items)

    spy = Spy(ctx, keys)
    boot.bootstrap(spy, spy.mod_drop(spy.encrypt(np.zeros(4), 1), 0), bp)
    assert set(used) <= set(steps) and ckks.STEP_CONJUGATE in used
    assert any(t not in (0, ckks.STEP_CONJUGATE) and abs(t) >= 8 for t in used)  # giant steps seen


def _centered(r, q):
    q = np.asarray(q, np.int64).reshape(-1, 1)
    v = r.astype(np.int64) % q
    return np.where(v > q // 2, v - q, v)


def test_rotate_sum_is_the_sum_of_rotations_up_to_moddown_rounding(boot11):
    """One ModDown for a sum of rotations differs from the sum of the
    separate rotations only by the rounding of the divisions by P: the
    difference of every component is one small integer polynomial (the same
    integer in every limb), at most (alpha + 1) per rotated term."""
    bs, p, ctx, bp, keys, ev = boot11
    rng = np.random.default_rng(11)
    steps = [0] + [t for t in boot.rotation_steps(bs.logN, bp) if t != ckks.STEP_CONJUGATE][:4]
    for l in (p.L, p.top_level, 2):
        items = []
        for i, t in enumerate(steps):
            z = rng.uniform(-1, 1, p.slots)
            ct = ev.mod_drop(ev.encrypt(z, 40 + i), min(l, p.top_level))
            if l > p.top_level:
                ct = ckks.Ciphertext(l, np.array([rng.integers(0, int(ctx.q[j]), p.N, dtype=np.uint64)
                                                  for j in range(l + 1)]),
                                     np.array([rng.integers(0, int(ctx.q[j]), p.N, dtype=np.uint64)
                                               for j in range(l + 1)]))
            items.append((ct, t))
        got = ev.rotate_sum(items)
        ref = None
        for ct, t in items:
            r = ev.rotate(ct, t)
            ref = r if ref is None else ev.add(ref, r)
        assert got.level == ref.level == l
        k = sum(1 for _, t in items if t)
        for a, b in ((got.c0, ref.c0), (got.c1, ref.c1)):
            d = _centered(a.astype(np.int64) - b.astype(np.int64), ctx.q[: l + 1])
            assert (d == d[0]).all()
            assert np.abs(d[0]).max() <= k * (p.alpha + 1)
        if l <= p.top_level:
            assert np.abs(ev.decrypt(got, p.slots) - ev.decrypt(ref, p.slots)).max() < 1e-6


def test_hoisted_moddown_linear_transform_matches_separate_rotations(boot11):
    """A CoeffToSlot group with its giant steps sharing one ModDown decrypts
    to the same slots as with one rotation per giant step."""
    bs, p, ctx, bp, keys, ev = boot11
    z = synth.boot_inputs(bs, 1)[0]
    x = ev.encrypt(z, 5)
    st = boot.stage_groups(bs.logN - 1, bs.cts, ascending=False)[0]
    D = boot.group_diagonals(bs.logN, st, True, 1.0)
    a = boot.linear_transform(ev, x, D, 1 << min(st), x.level - 1, hoist=True)
    b = boot.linear_transform(ev, x, D, 1 << min(st), x.level - 1, hoist=False)
    assert a.level == b.level == x.level - 1
    assert np.abs(ev.decrypt_c(a, p.slots) - ev.decrypt_c(b, p.slots)).max() < 1e-7


def test_deep_composite_brings_the_circuit_within_1e2_of_the_exact_kan():
    """Bootstrapping lets a layer spend its levels on a deep comparison: with
    f_3 four times (depth 12) the HE-friendly tiny network is within 1e-2 of
    the exact KAN, where the 7-level layers' f_1 is not; its layers take 17
    levels, which boot11deep keeps between refreshes (slot simulator)."""
    from oracle import circuit, kan
    from oracle.slotsim import SlotSim
    wl = synth.WORKLOADS["tinydeep"]
    raw = synth.raw_weights(wl)
    x = synth.inputs(wl, 200)
    deep = kan.compile_model(raw, synth.calibration_inputs(wl, 512), [wl.silu_degree] * 2,
                             [list(c) for c in wl.comp_degrees], wl.grid, wl.silu_range, prescale=wl.prescale)
    shallow = kan.compile_model(raw, synth.calibration_inputs(wl, 512), [wl.silu_degree] * 2, [[3], [3]], wl.grid,
                                wl.silu_range, prescale=False)
    assert np.abs(kan.he_friendly_kan(x, deep) - kan.exact_kan(x, deep)).max() < 1e-2
    assert np.abs(kan.he_friendly_kan(x, shallow) - kan.exact_kan(x, shallow)).max() > 0.1
    bs = synth.BOOTSETS["boot11deep"]
    sim = SlotSim(1 << (bs.logN - 1))
    ct = sim.fresh(x[0], bs.Lc)
    y, nb = circuit.layer_forward(sim, [ct], deep[0], 0, True)
    assert y.level >= 0
    y2, _ = circuit.layer_forward(sim, [sim.fresh(y.v, bs.Lc)], deep[1], nb, False)
    assert y2.level >= 0 and bs.Lc - y.level == 17


@pytest.fixture(scope="module")
def boot11_real(boot11):
    bs, p, ctx, bp, keys, ev = boot11
    return bs, p, ctx, boot.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree, real_slots=True), keys, ev


@pytest.mark.parametrize("n", [8, 64, 256])
def test_sparse_refresh_keeps_a_periodic_message(boot11, n):
    """A sparsely packed refresh (slots n: SubSum, then the transforms' first
    log2 n stages) of a message whose slots repeat with period n decrypts to
    it, periodic, with fewer key switches than the full-slot refresh; and the
    CoeffToSlot output holds the sparse plaintext's coefficients over 2 q_0
    (near integers plus m / (2 q_0), within [-K/2, K/2])."""
    bs, p, ctx, bp_full, _, _ = boot11
    M = p.slots
    bp = boot.make_params(2 if n > 8 else 1, 2 if n > 8 else 1, bs.K, bs.r, bs.degree, slots=n)
    keys = ckks.Keys(ctx, synth.SEED_KEYGEN, boot.rotation_steps(bs.logN, bp))
    ev = ckks.Oracle(ctx, keys)
    z = np.tile(np.random.default_rng(n).uniform(-1, 1, n), M // n)
    ct = ev.encrypt(z, 22)
    want = ev.decrypt(ct, p.slots)
    tr = {}
    out = boot.bootstrap(ev, ct, bp, tr)
    assert out.level == p.top_level
    got = ev.decrypt_c(out, p.slots)
    assert np.abs(got.real - want).max() < 1e-6 and np.abs(got.imag).max() < 1e-6
    assert np.abs(got.real - np.tile(got.real[:n], M // n)).max() < 1e-7
    assert ev.count["ks"] < 79  # the full-slot refresh of boot11: 79 key switches
    w = decrypt_wide(ev, tr["cts"])
    assert np.abs(w.real).max() <= bs.K / 2 and np.abs(w.imag).max() <= bs.K / 2
    assert np.abs(2 * w.real - np.round(2 * w.real)).max() < 1e-3
    # the real-slot variant (SlotToCoeff first, also sparse) of the same input
    rbp = boot.make_params(1, 1, bs.K, bs.r, bs.degree, real_slots=True, slots=n)
    rev = ckks.Oracle(ctx, ckks.Keys(ctx, synth.SEED_KEYGEN, boot.rotation_steps(bs.logN, rbp)))
    rct = rev.mod_drop(rev.encrypt(z, 23), 1)
    rout = boot.bootstrap(rev, rct, rbp)
    assert rout.level == p.top_level
    assert np.abs(rev.decrypt(rout, p.slots) - rev.decrypt(rct, p.slots)).max() < 1e-6
    with pytest.raises(ValueError):
        boot.bootstrap(ev, ct, boot.make_params(1, 1, bs.K, bs.r, bs.degree, slots=n + 1))


def test_real_slot_refresh_with_slot_to_coeff_first(boot11_real):
    """SlotToCoeff first: its output's low coefficients are c1 S R z (exactly
    the slots, bit-reversed, up to rounding); the refresh decrypts to the
    input's real parts from the lowest allowed level and from the top, with
    one EvalMod and fewer key switches than the full refresh."""
    bs, p, ctx, bp, keys, ev = boot11_real
    z = synth.boot_inputs(bs, 1, stream=7)[0]
    m = p.logN - 1
    R = np.array([int(format(i, "0%db" % m)[::-1], 2) for i in range(p.slots)])
    for lvl in (bs.stc, p.top_level):
        ct = ev.mod_drop(ev.encrypt(z, 31), lvl)
        tr = {}
        before = dict(ev.count)
        out = boot.bootstrap(ev, ct, bp, tr)
        ks = ev.count["ks"] - before["ks"]
        x = tr["stc_first"]
        c = ev.phase(x).astype(object)
        q0 = int(ctx.q[0])
        coef = np.array([int(v) - q0 if int(v) > q0 // 2 else int(v) for v in c], dtype=np.float64)
        S = ctx.S[x.level]
        assert np.abs(coef[:p.slots] / (S * boot.REAL_C1) - z[R]).max() < 1e-4
        assert np.abs(coef[p.slots:] / (S * boot.REAL_C1)).max() < 1e-4
        got = ev.decrypt_c(out, p.slots)
        assert out.level == p.top_level
        assert np.abs(got.real - ev.decrypt(ct, p.slots)).max() < 1e-6 and np.abs(got.imag).max() < 1e-6
    full = dict(ev.count)
    boot.bootstrap(ev, ev.mod_drop(ev.encrypt(z, 32), 1), boot.make_params(bs.cts, bs.stc, bs.K, bs.r, bs.degree))
    assert ks < ev.count["ks"] - full["ks"]
    with pytest.raises(ValueError):
        boot.bootstrap(ev, ev.mod_drop(ev.encrypt(z, 33), bs.stc - 1), bp)
