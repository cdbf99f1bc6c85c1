"""CKKS bootstrapping on the oracle's RNS-CKKS: the ciphertext refresh the
paper's Experiment Setup relies on (multiplicative depth 20 with
bootstrapping in the settings of Lee et al. 2022).  The paper gives no
procedure of its own, so the reading here is the standard full-slot RNS-CKKS
bootstrapping (Cheon, Han, Kim, Kim, Song 2018; Chen, Chillotti, Song 2019;
Han, Ki 2020) on a chain whose top `boot_levels` primes are wide.

TEST INFRASTRUCTURE ONLY: used by tests/ and the golden-value scripts; never
by the product package.

With M = N/2 slots, m = log2 M, zeta = exp(i pi / N) and the special DFT of
the encoding U0[j][k] = zeta^(5^j k) (j, k < M), a plaintext polynomial t has
slots tau(t) = U0 (t_lo + i t_hi), t_lo/t_hi its low/high N/2 coefficients.
U0 factors as F_{m-1} ... F_0 R: R the bit reversal of m-bit indices and F_s
the butterfly stage of half-width h = 2^s, which maps v to
  out_p = v_p + w_s(p mod h) v_{p+h}          (bit s of p clear)
  out_p = v_{p-h} - w_s(p mod h) v_p          (bit s of p set)
with w_s(j) = exp(2 pi i (5^j mod 8h) / (8h)) = zeta^((5^j mod 8h) M / (2h)).

bootstrap(ct) at level l (a computation level):
  1. ModRaise: the residues mod q_0, read as centred integers, lifted to the
     top level L; the plaintext becomes t = m + q_0 I, I small (|I| <= K).
  2. CoeffToSlot: multiply the slots tau(t)/S_L by
     (S_L / (2 q_0)) (2/N) U0^H = (S_L / (2 q_0)) R (F_0^H/2) ... (F_{m-1}^H/2);
     R is left out (SlotToCoeff starts from the bit-reversed order), so the
     slots hold R (t_lo + i t_hi) / (2 q_0).  The stages run in cts_levels
     groups of consecutive stages; each group is one product by the diagonals
     of its merged matrix (baby-step giant-step rotations, one level).
  3. Split: y_lo = w + conj(w) holds R t_lo / q_0, y_hi = i (conj(w) - w)
     holds R t_hi / q_0 (conj: the Galois element 2N-1; i: the monomial
     X^(N/2)).
  4. EvalMod on each: the Chebyshev series of cos(2 pi (y - 1/4) / 2^r) on
     [-K, K], then r double-angle steps c <- 2 c^2 - 1, giving
     cos(2 pi (y - 1/4)) = sin(2 pi y) ~ 2 pi m_k / q_0 (|m_k| << q_0).
  5. Recombine u_lo + i u_hi, then SlotToCoeff: F_{m-1} ... F_0 times
     q_0 / (2 pi S_l) in stc_levels groups (F_0 first), the last group landing
     at the top computation level: the slots hold tau(m) / S_l, the input's
     slot values.
Sparse packing (slots = n < N/2, a power of two; Cheon, Han, Kim, Kim, Song
2018): a message whose slot vector repeats with period n is a polynomial in
Y = X^(N/(2n)) of degree < 2n, with n slots of its own at the powers of
zeta' = zeta^(N/(2n)).  For s < log2 n the stage F_s pairs indices inside
aligned blocks of n and its twiddles are those of the n-slot factorisation
(zeta^((5^j mod 8h) M/(2h)) = zeta'^((5^j mod 8h) n/(2h))), so the first
log2 n stages act on every block as the n-slot transform.  After ModRaise,
t = m + q_0 I is a full polynomial again; SubSum, the sum of the rotations by
n 2^k (k < log2(M/n)), keeps its monomials in Y times M/n and makes the slots
n-periodic; CoeffToSlot then runs the first log2 n stages only, its constant
times n/M, and SlotToCoeff likewise (steps 3 to 5 unchanged).
Every merged diagonal entry is one path through the butterflies, so it is
sign * 2^-(stages, CoeffToSlot only) * zeta^e exactly; its parts are the
doubles nearest zeta^e's, scaled by the power of two and the sign (exact),
then multiplied by the group's constant (one rounding).  The baby-step width
of a group whose offsets are multiples of u is b1 = u 2^ceil(log2 b), b the
least integer with b^2 >= 2 R/u + 1 (R the largest |offset|); offset
o = g b1 + b' with g = floor(o / b1).
"""
import dataclasses
import math

import numpy as np

from . import ckks
from .circuit import cheb_eval, pow2ceil


@dataclasses.dataclass(frozen=True)
class BootParams:
    """cts_levels / stc_levels: stage groups (levels) of CoeffToSlot and
    SlotToCoeff; K: EvalMod's input range [-K, K]; r: double-angle steps;
    coeffs: Chebyshev coefficients of cos(2 pi (y - 1/4) / 2^r) on [-K, K];
    real_slots: refresh real slot values with SlotToCoeff first (below);
    hoist_moddown: the giant steps of each baby-step giant-step product
    share one ModDown (linear_transform); slots: n, the period of the slot
    vector a sparse refresh keeps (a power of two below N/2; 0: all N/2
    slots)."""
    cts_levels: int
    stc_levels: int
    K: float
    r: int
    coeffs: tuple
    real_slots: bool = False
    hoist_moddown: bool = True
    slots: int = 0


# SlotToCoeff-first refresh: the coefficients it writes are c1 times the slots
REAL_C1 = 2.0 ** -7


def cos_coeffs(K, r, degree):
    """Chebyshev interpolant of cos(2 pi (y - 1/4) / 2^r) on [-K, K] at the
    degree+1 Chebyshev nodes: c_k = (2/n) sum_j f(K cos th_j) cos(k th_j),
    th_j = pi (j + 1/2) / n, c_0 halved."""
    n = degree + 1
    th = np.pi * (np.arange(n) + 0.5) / n
    f = np.cos(2.0 * np.pi * (K * np.cos(th) - 0.25) / 2.0 ** r)
    c = np.array([2.0 / n * np.sum(f * np.cos(k * th)) for k in range(n)])
    c[0] *= 0.5
    return tuple(float(v) for v in c)


def make_params(cts_levels, stc_levels, K, r, degree, real_slots=False, hoist_moddown=True, slots=0):
    return BootParams(cts_levels, stc_levels, float(K), r, cos_coeffs(K, r, degree), real_slots, hoist_moddown,
                      slots)


def slot_stages(logN, bp):
    """(n, log2 n): the slots a refresh keeps and the butterfly stages its
    transforms run"""
    M = 1 << (logN - 1)
    n = bp.slots or M
    if n & (n - 1) or not 2 <= n <= M:
        raise ValueError("slots must be a power of two between 2 and N/2")
    return n, n.bit_length() - 1


def subsum_steps(logN, bp):
    """the rotation steps of SubSum: n 2^k for k < log2(M/n)"""
    M = 1 << (logN - 1)
    n, _ = slot_stages(logN, bp)
    return [n << k for k in range((M // n).bit_length() - 1)]


def evalmod_plain(y, bp):
    """EvalMod in FP64 on plain values (the series, then the double angles)."""
    u = np.clip(np.asarray(y, np.float64) / bp.K, -1.0, 1.0)
    c = np.polynomial.chebyshev.chebval(u, bp.coeffs)
    for _ in range(bp.r):
        c = 2.0 * c * c - 1.0
    return c


def stage_groups(m, G, ascending):
    """m butterfly stages in G groups of consecutive stages, in application
    order (ascending: F_0 first, SlotToCoeff; descending: F_{m-1} first,
    CoeffToSlot); group sizes m // G, the first m % G groups one larger."""
    if not 1 <= G <= m:
        raise ValueError("stage groups must be between 1 and log2(N/2)")
    order = list(range(m)) if ascending else list(range(m - 1, -1, -1))
    out, pos = [], 0
    for g in range(G):
        n = m // G + (1 if g < m % G else 0)
        out.append(order[pos:pos + n])
        pos += n
    return out


def twiddle_exponents(s, M):
    """e_j with zeta^(e_j) = w_s(j), j < 2^s: (5^j mod 8h) M / (2h)."""
    h = 1 << s
    e = np.empty(h, np.int64)
    v = 1
    for j in range(h):
        e[j] = v * (M // (2 * h))
        v = v * 5 % (8 * h)
    return e


def group_terms(logN, stages, inverse):
    """Every non-zero entry (row i, column j) of the product of the stages
    (applied in list order) as arrays i, j, sign, e: the entry is
    sign * zeta^e, times 2^-len(stages) when inverse (F_s^H / 2)."""
    N = 1 << logN
    M, twoN = N // 2, 2 * N
    tw = {s: twiddle_exponents(s, M) for s in stages}
    gmask = sum(1 << s for s in stages)
    i = np.arange(M, dtype=np.int64)
    I, J, SG, E = [], [], [], []
    for c in range(1 << len(stages)):
        j = i & ~gmask
        for k, s in enumerate(stages):
            if c >> k & 1:
                j = j | (1 << s)
        p = j.copy()
        sg = np.ones(M, np.int64)
        e = np.zeros(M, np.int64)
        for s in stages:
            h = 1 << s
            q = p
            p = (p & ~h) | (i & h)
            qs, ps = (q >> s) & 1, (p >> s) & 1
            w = tw[s][p & (h - 1)]
            if inverse:
                sg = sg * np.where((ps == 1) & (qs == 1), -1, 1)
                e = (e + np.where(ps == 1, twoN - w, 0)) % twoN
            else:
                sg = sg * np.where((qs == 1) & (ps == 1), -1, 1)
                e = (e + np.where(qs == 1, w, 0)) % twoN
        I.append(i)
        J.append(j)
        SG.append(sg)
        E.append(e)
    return np.concatenate(I), np.concatenate(J), np.concatenate(SG), np.concatenate(E)


_roots = {}


def root_table(logN):
    """the doubles nearest the parts of zeta^e, e < 2N"""
    if logN not in _roots:
        N = 1 << logN
        re = np.zeros(2 * N)
        im = np.zeros(2 * N)
        ckks.lib().oc_root_table(logN, ckks.P(re), ckks.P(im))
        _roots[logN] = (re, im)
    return _roots[logN]


def group_diagonals(logN, stages, inverse, const):
    """{offset o in (-M/2, M/2]: (re, im)} with diag_o[i] = entry (i, i+o mod M)
    of the group's matrix times const."""
    N = 1 << logN
    M = N // 2
    I, J, SG, E = group_terms(logN, stages, inverse)
    rre, rim = root_table(logN)
    f = SG.astype(np.float64) * (0.5 ** len(stages) if inverse else 1.0)
    re = (f * rre[E]) * const
    im = (f * rim[E]) * const
    o = (J - I) % M
    o = np.where(o > M // 2, o - M, o)
    out = {}
    for off in np.unique(o):
        sel = o == off
        dre = np.zeros(M)
        dim = np.zeros(M)
        dre[I[sel]] = re[sel]
        dim[I[sel]] = im[sel]
        out[int(off)] = (dre, dim)
    return out


def bsgs_width(offsets, u):
    R = max(abs(o) for o in offsets) // u
    b = 1
    while b * b < 2 * R + 1:
        b += 1
    return u * pow2ceil(b)


def linear_transform(ev, x, diags, u, t, hoist=True):
    """sum_o diag_o * rot(x, o) at level t by baby-step giant-step:
    sum_g rot( sum_b rot(diag_(g b1 + b), -g b1) * rot(x, b), g b1 ).
    hoist: the giant-step rotations share one ModDown (Oracle.rotate_sum);
    else each giant step is a rotation of its own, added in giant order."""
    offs = sorted(diags)
    b1 = bsgs_width(offs, u)
    giants = sorted(set(o // b1 for o in offs))
    babies = sorted(set(o - (o // b1) * b1 for o in offs))
    xd = ev.mod_drop(x, t + 1)
    rots = {b: (xd if b == 0 else ev.rotate(xd, b)) for b in babies}
    z = None
    items = []
    for g in giants:
        terms = []
        for b in babies:
            o = g * b1 + b
            if o not in diags:
                continue
            re, im = diags[o]
            v = np.empty(len(re), np.complex128)
            v.real = np.roll(re, g * b1)
            v.imag = np.roll(im, g * b1)
            terms.append((rots[b], v))
        inner = ev.lincomb(terms, t)
        if hoist:
            items.append((inner, g * b1))
            continue
        if g:
            inner = ev.rotate(inner, g * b1)
        z = inner if z is None else ev.add(z, inner)
    return ev.rotate_sum(items) if hoist else z


def transform_plan(logN, bp, S_top, q0, S_in):
    """[(stages, inverse, const)] for CoeffToSlot then SlotToCoeff (a sparse
    refresh: the first log2 n stages, CoeffToSlot's constant times n/M for
    SubSum's factor M/n)."""
    n, m = slot_stages(logN, bp)
    sub = n / float(1 << (logN - 1))
    plan = []
    for gi, st in enumerate(stage_groups(m, bp.cts_levels, ascending=False)):
        plan.append((st, True, S_top / (2.0 * float(q0)) * sub if gi == 0 else 1.0))
    for gi, st in enumerate(stage_groups(m, bp.stc_levels, ascending=True)):
        plan.append((st, False, float(q0) / (2.0 * math.pi * S_in) if gi == 0 else 1.0))
    return plan


def rotation_steps(logN, bp):
    """every rotation step the bootstrapping uses, with STEP_CONJUGATE"""
    _, m = slot_stages(logN, bp)
    steps = {ckks.STEP_CONJUGATE} | set(subsum_steps(logN, bp))
    for st, inv in [(g, True) for g in stage_groups(m, bp.cts_levels, False)] + \
                   [(g, False) for g in stage_groups(m, bp.stc_levels, True)]:
        I, J, _, _ = group_terms(logN, st, inv)
        M = 1 << (logN - 1)
        o = (J - I) % M
        o = np.where(o > M // 2, o - M, o)
        offs = sorted(set(int(v) for v in np.unique(o)))
        b1 = bsgs_width(offs, 1 << min(st))
        for v in offs:
            g = v // b1
            if v - g * b1:
                steps.add(v - g * b1)
            if g:
                steps.add(g * b1)
    return sorted(steps)


def eval_mod(ev, y, bp):
    c = cheb_eval(ev, y, list(bp.coeffs), -bp.K, bp.K)
    for _ in range(bp.r):
        c = ev.add_const(ev.mul_int(ev.mul(c, c), 2), -1.0)
    return c


def bootstrap_real(ev, ct, bp, trace=None):
    """Refresh of real slot values with SlotToCoeff first (Chen, Chillotti,
    Song 2019: the special DFT runs on the input, at its own few limbs):
      1. F_{m-1} ... F_0 times c1 on the slots z (stc_levels groups, F_0 first,
         landing stc_levels below the input): the plaintext's low N/2
         coefficients become S c1 R z (S the scale there; high half: the
         imaginary parts, zero for real z);
      2. ModRaise and CoeffToSlot as in the full refresh: the slots hold
         (R t_lo + i R t_hi) / (2 q_0) with R t_lo = S c1 z + q_0 R I_lo;
      3. y = w + conj(w) = S c1 z / q_0 + integers; EvalMod gives
         sin(2 pi y) ~ 2 pi S c1 z / q_0 (one EvalMod: the imaginary half,
         which holds no message, is dropped);
      4. one product by q_0 / (2 pi S c1) lands at the top computation level.
    The input must hold stc_levels levels; the result's slots are Re z.  A
    sparse refresh (slots n) runs the first log2 n stages in steps 1 and 2,
    with SubSum after ModRaise and CoeffToSlot's constant times n/M, as in
    bootstrap."""
    ctx, p = ev.ctx, ev.ctx.p
    n, m = slot_stages(p.logN, bp)
    if ct.level > p.top_level or ct.level < bp.stc_levels:
        raise ValueError("real-slot bootstrapping input must be at a computation level >= stc_levels")
    x = ct
    for gi, st in enumerate(stage_groups(m, bp.stc_levels, ascending=True)):
        x = linear_transform(ev, x, group_diagonals(p.logN, st, False, REAL_C1 if gi == 0 else 1.0), 1 << min(st),
                             x.level - 1, bp.hoist_moddown)
    if trace is not None:
        trace["stc_first"] = x
    lp = x.level
    x = ev.mod_raise(ev.mod_drop(x, 0))
    for t in subsum_steps(p.logN, bp):
        x = ev.add(x, ev.rotate(x, t))
    sub = n / float(p.slots)
    for gi, st in enumerate(stage_groups(m, bp.cts_levels, ascending=False)):
        cst = float(ctx.S[p.L]) / (2.0 * float(ctx.q[0])) * sub if gi == 0 else 1.0
        x = linear_transform(ev, x, group_diagonals(p.logN, st, True, cst), 1 << min(st), x.level - 1,
                             bp.hoist_moddown)
    if trace is not None:
        trace["cts"] = x
    y = ev.add(x, ev.rotate(x, ckks.STEP_CONJUGATE))
    u = eval_mod(ev, y, bp)
    if trace is not None:
        trace["evalmod"] = u
    if u.level <= p.top_level:
        raise ValueError("bootstrapping does not fit the boot levels")
    return ev.lincomb([(u, float(ctx.q[0]) / (2.0 * math.pi * float(ctx.S[lp]) * REAL_C1))], p.top_level)


def bootstrap(ev, ct, bp, trace=None):
    """The refreshed ciphertext at the top computation level (steps above).
    trace: optional dict receiving the intermediate ciphertexts."""
    slot_stages(ev.ctx.p.logN, bp)
    if bp.real_slots:
        return bootstrap_real(ev, ct, bp, trace)
    ctx, p = ev.ctx, ev.ctx.p
    if ct.level > p.top_level:
        raise ValueError("bootstrapping input above the top computation level")
    plan = transform_plan(p.logN, bp, float(ctx.S[p.L]), int(ctx.q[0]), float(ctx.S[ct.level]))
    x = ev.mod_raise(ev.mod_drop(ct, 0))
    if trace is not None:
        trace["raised"] = x
    for t in subsum_steps(p.logN, bp):
        x = ev.add(x, ev.rotate(x, t))
    for st, inv, cst in plan[:bp.cts_levels]:
        x = linear_transform(ev, x, group_diagonals(p.logN, st, inv, cst), 1 << min(st), x.level - 1,
                             bp.hoist_moddown)
    if trace is not None:
        trace["cts"] = x
    xc = ev.rotate(x, ckks.STEP_CONJUGATE)
    y_lo = ev.add(x, xc)
    y_hi = ev.mul_i(ev.sub(xc, x))
    if trace is not None:
        trace["conj"] = xc
        trace["split"] = (y_lo, y_hi)
    u_lo = eval_mod(ev, y_lo, bp)
    u_hi = eval_mod(ev, y_hi, bp)
    if trace is not None:
        trace["evalmod"] = (u_lo, u_hi)
    w = ev.add(u_lo, ev.mul_i(u_hi))
    if trace is not None:
        trace["recombined"] = w
    stc = plan[bp.cts_levels:]
    for gi, (st, inv, cst) in enumerate(stc):
        t = p.top_level if gi == len(stc) - 1 else w.level - 1
        if t < p.top_level or t >= w.level:
            raise ValueError("bootstrapping does not fit the boot levels")
        w = linear_transform(ev, w, group_diagonals(p.logN, st, inv, cst), 1 << min(st), t, bp.hoist_moddown)
    return w
