"""The encrypted KAN circuit on the oracle's RNS-CKKS (O1 running O2's math).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.

Per KANLayer (Method, Figure 2 structure) on a ciphertext x whose slots hold
the layer input in blocks of n_blk slots, in the paper's order (`PAPER`):
  * first layer: Fast Repeat Packing (Algorithm 1) without the mask, because
    a fresh ciphertext already holds zeros outside [0, n_i);
  * spline branch, Algorithm 2 as written: PolyComp on (x_rep - g1)/2R and on
    (g2 - x_rep)/2R, their product, and k rounds of the order recursion (each
    round relinearises once after summing both tensor products);
  * SiLU branch: the fitted Chebyshev polynomial by baby-step giant-step on x;
  * the two linear layers as two products, W_f = W' P (Lazy Combination,
    Algorithm 3) with the bases and W_b with the SiLU values, each by the
    hybrid diagonal method with baby-step giant-step rotations and a fold
    over all slots, so each output is periodic with period d = next power of
    two >= n_out (the next layer's repeat packing comes for free); the layer
    output is their sum.
Four restructurings (`Circuit`) change no value of the FP64 circuit and cut
key switches or their ModDowns; each is a named option, checked against the
paper's order:
  * shared_comparison: when the input holds g+2k+1 blocks, the second
    comparison S((t_{m+2} - x)/2R) is 1 - S((x - t_{m+2})/2R) (the composite
    is odd), i.e. 1 minus the first comparison of block m+1: one rotation
    instead of a second PolyComp;
  * fused_linear: the SiLU branch runs on the repeat-packed input with its
    coefficients masked to block g+k (the first block the bases leave free)
    and is added to the bases, so one product with [W_f | W_b] and one fold
    compute both linear layers;
  * folded_period: a hidden layer's block layout repeats with the shortest
    power-of-two period that holds its blocks, and the fold runs over one
    period;
  * shared_moddown: the giant-step rotations of each baby-step giant-step
    product share one ModDown (Oracle.rotate_sum: their key-switch
    accumulators are added over Q_l u P and divided by P once), which changes
    the residues by the rounding of those divisions only;
  * a first layer whose repeat-packed footprint n_i 2^ceil(log2(g+2k))
    exceeds the slot count takes its input as several ciphertexts, one per
    chunk of consecutive features: each chunk is packed and expanded on its
    own and multiplied by its columns of W_b and W_f, and the chunks' partial
    sums are added before the single fold;
  * S input vectors may share a ciphertext (S a power of two): feature i of
    vector s sits in slot i S + s, every block is S times wider, and the
    linear layers act as W (x) I_S, whose only non-zero generalised diagonals
    are the multiples of S, so the rotations are S times longer but as many;
    outputs are periodic with period d S.
Every step fixes where rescales happen and at which scale each plaintext is
encoded, which the GPU path reproduces independently.
"""
import dataclasses
import math

import numpy as np

from .kan import fused_weights, lazy_weights


@dataclasses.dataclass(frozen=True)
class Circuit:
    """Which restructurings of the paper's circuit are applied (all off: the
    paper's order).  naive_permutation is the comparison method of the
    paper's basis-approximation experiments instead: no lazy combination of
    the permutation, the bases are permuted from ColTile order into row order
    by a homomorphic permutation and multiplied by W' itself (it excludes
    fused_linear and folded_period)."""
    shared_comparison: bool = False
    fused_linear: bool = False
    folded_period: bool = False
    naive_permutation: bool = False
    shared_moddown: bool = False


PAPER = Circuit()
RESTRUCTURED = Circuit(True, True, True, False, True)


def pow2ceil(n):
    return 1 << max(0, (n - 1).bit_length())


def clog2(n):
    return max(0, (n - 1).bit_length())


# --------------------------------------------------------------------------
# polynomial evaluators
# --------------------------------------------------------------------------
def odd_poly(ev, v, a):
    """sum_i a_i v^(2i+1) for degree 3, 5 or 7 in depth 2, 3, 3."""
    l = v.level
    if len(a) == 2:
        v2 = ev.mul(v, v)
        t3 = ev.mul(ev.lincomb([(v, a[1])], l - 1), v2)
        return ev.add(ev.lincomb([(v, a[0])], l - 2), t3)
    if len(a) == 3:
        v2 = ev.mul(v, v)
        v4 = ev.mul(v2, v2)
        t3 = ev.mul(ev.lincomb([(v, a[1])], l - 1), v2)
        t5 = ev.mul(ev.lincomb([(v, a[2])], l - 2), v4)
        return ev.add(ev.lincomb([(v, a[0]), (t3, 1.0)], l - 3), t5)
    if len(a) == 4:
        v2 = ev.mul(v, v)
        v4 = ev.mul(v2, v2)
        t3 = ev.mul(ev.lincomb([(v, a[1])], l - 1), v2)
        t7 = ev.mul(ev.lincomb([(v, a[3])], l - 1), v2)
        B = ev.add(t7, ev.lincomb([(v, a[2])], l - 2))
        Cc = ev.mul(B, v4)
        return ev.add(ev.lincomb([(v, a[0]), (t3, 1.0)], l - 3), Cc)
    raise ValueError("odd polynomial of unsupported degree")


def polycomp(ev, v, stages):
    """PolyComp(v, 0) = (F(v/2R)+1)/2 with the scalings folded into the stages."""
    for a in stages:
        v = odd_poly(ev, v, list(a))
    return ev.add_const(v, 0.5)


def cheb_split(c, G):
    """p = q T_G + r for Chebyshev coefficients c (len n <= 2G):
    q_0 = c_G, q_j = 2 c_{G+j}; r_i = c_i, r_{G-j} -= c_{G+j}  (j >= 1)."""
    n = len(c)
    q = [c[G]] + [2.0 * c[G + j] for j in range(1, n - G)]
    r = list(c[:G])
    for j in range(1, n - G):
        r[G - j] = r[G - j] - c[G + j]
    return q, r


class ChebEval:
    """Chebyshev series on [lo, hi] by baby-step giant-step.

    T_1 = alpha x + beta (one rescale), babies T_2..T_b with
    T_2i = 2 T_i^2 - 1 and T_2i+1 = 2 T_i T_{i+1} - T_1, giants
    T_2b, T_4b, ... by squaring; the series is split recursively by the
    largest giant below its length, and every sub-result lands exactly on the
    level its consumer needs (leaf lincombs target that level directly)."""

    def __init__(self, ev, x, coeffs, lo, hi, mask=None):
        self.ev = ev
        self.mask = mask  # None, or a slot vector every coefficient is multiplied by
        self.c = [float(v) for v in coeffs]
        deg = len(self.c) - 1
        m = clog2(deg + 1)
        self.b = 1 << ((m + 1) // 2)
        alpha = 2.0 / (hi - lo)
        beta = -(hi + lo) / (hi - lo)
        T1 = ev.add_const(ev.lincomb([(x, alpha)], x.level - 1), beta)
        T = {1: T1}
        for i in range(2, self.b + 1):
            if i % 2 == 0:
                h = T[i // 2]
                T[i] = ev.add_const(ev.mul_int(ev.mul(h, h), 2), -1.0)
            else:
                a, c = T[(i - 1) // 2], T[(i + 1) // 2]
                lv = min(a.level, c.level)
                p = ev.mul_int(ev.mul(ev.level_down(a, lv), ev.level_down(c, lv)), 2)
                T[i] = ev.sub(p, ev.level_down(T1, p.level))
        G = 2 * self.b
        while G < deg + 1:
            h = T[G // 2]
            T[G] = ev.add_const(ev.mul_int(ev.mul(h, h), 2), -1.0)
            G *= 2
        self.T = T

    def giant(self, n):
        G = self.b
        while 2 * G < n:
            G *= 2
        return G

    def feasible(self, c, t):
        n = len(c)
        if n <= self.b:
            return t <= min(self.T[i].level for i in range(1, n)) - 1
        G = self.giant(n)
        q, r = cheb_split(c, G)
        if len(q) == 1:
            ok_q = t <= self.T[G].level - 1
        else:
            ok_q = t + 1 <= self.T[G].level and self.feasible(q, t + 1)
        return ok_q and self.feasible(r, t)

    def coef(self, v):
        return v if self.mask is None else v * self.mask

    def rec(self, c, t):
        ev = self.ev
        n = len(c)
        if n <= self.b:
            terms = [(self.T[i], self.coef(c[i])) for i in range(1, n)]
            s = ev.lincomb(terms, t)
            return ev.add_const(s, c[0]) if self.mask is None else ev.add_vec(s, c[0] * self.mask)
        G = self.giant(n)
        q, r = cheb_split(c, G)
        if len(q) == 1:
            prod = ev.lincomb([(self.T[G], self.coef(q[0]))], t)
        else:
            qc = self.rec(q, t + 1)
            prod = ev.mul(qc, ev.level_down(self.T[G], t + 1))
        return ev.add(prod, self.rec(r, t))

    def run(self):
        t = self.T[1].level - 1
        while not self.feasible(self.c, t):
            t -= 1
            if t < 0:
                raise RuntimeError("Chebyshev evaluation does not fit the level budget")
        return self.rec(self.c, t)


def cheb_eval(ev, x, coeffs, lo, hi, mask=None):
    """The series on every slot of x; with a mask, every coefficient (and so
    the result) is multiplied slot-wise by it, at no extra depth."""
    return ChebEval(ev, x, coeffs, lo, hi, mask).run()


# --------------------------------------------------------------------------
# packing, B-spline bases, linear layers
# --------------------------------------------------------------------------
def repeat_pack(ev, x, n_blk, nlog):
    """Algorithm 1 without the mask: x <- rot(x, -n_blk 2^(j-1)) + x."""
    for j in range(1, nlog + 1):
        x = ev.add(ev.rotate(x, -n_blk * (1 << (j - 1))), x)
    return x


def coltile(knots, lo, hi, n_blk, n_in, slots, period=None):
    """ColTile(G, lo, hi) of the knot matrix G (row i = t_1..t_r for every
    input): block m (m < hi-lo) holds t_{lo+m} in slots m n_blk + i, i < n_in;
    every other slot is 0; the layout repeats every `period` slots (default:
    once).  lo, hi are 1-based as in Algorithm 2."""
    period = slots if period is None else period
    v = np.zeros(period)
    for m in range(hi - lo):
        v[m * n_blk:m * n_blk + n_in] = knots[lo + m - 1]
    return np.tile(v, slots // period)


def block_mask(nblocks, n_blk, n_in, slots, period=None):
    period = slots if period is None else period
    v = np.zeros(period, bool)
    for m in range(nblocks):
        v[m * n_blk:m * n_blk + n_in] = True
    return np.tile(v, slots // period)


def bspline_basis(ev, xr, L, n_blk, width=None, shared=False, period=None):
    """Algorithm 2 on the repeat-packed ciphertext xr; `width` valid slots per
    block (n_in S when S vectors share the ciphertext).  shared: xr holds the
    input in g+2k+1 blocks, and the second comparison is taken from the first
    one: the composite is odd, so S((t_{m+2} - x)/2R) = 1 - S((x - t_{m+2})/2R),
    which is 1 minus the first comparison of block m+1 (one rotation instead
    of a second PolyComp).  period: the block layout repeats every `period`
    slots (the input must repeat likewise)."""
    slots = ev.ctx.p.slots
    width = L.n_in if width is None else width
    r = L.g + 2 * L.k + 1
    if shared:
        g1 = coltile(L.knots, 1, r + 1, n_blk, width, slots, period)  # t_1 .. t_r in blocks 0 .. r-1
        if L.comp_prescale:
            sc = L.comp_prescale
            x1 = polycomp(ev, ev.add_vec(ev.lincomb([(xr, sc)], xr.level - 1), -(g1 * sc)), L.comp)
        else:
            x1 = polycomp(ev, ev.add_vec(xr, -g1), L.comp)
        x2 = ev.add_const(ev.mul_int(ev.rotate(x1, n_blk), -1), 1.0)
    else:
        g1 = coltile(L.knots, 1, r, n_blk, width, slots, period)
        g2 = coltile(L.knots, 2, r + 1, n_blk, width, slots, period)
        if L.comp_prescale:
            # (x - g1) / 2R and (g2 - x) / 2R in one rescale each
            sc = L.comp_prescale
            x1 = polycomp(ev, ev.add_vec(ev.lincomb([(xr, sc)], xr.level - 1), -(g1 * sc)), L.comp)
            x2 = polycomp(ev, ev.add_vec(ev.lincomb([(xr, -sc)], xr.level - 1), g2 * sc), L.comp)
        else:
            x1 = polycomp(ev, ev.add_vec(xr, -g1), L.comp)
            x2 = polycomp(ev, ev.add_vec(ev.mul_int(xr, -1), g2), L.comp)
    b = ev.mul(x1, x2)
    for j in range(1, L.k + 1):
        nbl = r - j - 1
        t1 = coltile(L.knots, 1, r - j, n_blk, width, slots, period)
        t2 = coltile(L.knots, j + 1, r, n_blk, width, slots, period)
        t3 = coltile(L.knots, j + 2, r + 1, n_blk, width, slots, period)
        t4 = coltile(L.knots, 2, r - j + 1, n_blk, width, slots, period)
        msk = block_mask(nbl, n_blk, width, slots, period)
        A1 = np.zeros(slots)
        A2 = np.zeros(slots)
        A1[msk] = 1.0 / (t2[msk] - t1[msk])
        A2[msk] = 1.0 / (t3[msk] - t4[msk])
        lb = b.level
        P1 = ev.add_vec(ev.lincomb([(xr, A1)], lb), -(t1 * A1))
        P2 = ev.add_vec(ev.lincomb([(xr, -A2)], lb), t3 * A2)
        rb = ev.rotate(b, n_blk)
        b = ev.relin_rescale(ev.tensor_add(ev.tensor(P1, b), ev.tensor(P2, rb)))
    return b


def diag_vector(M, d, i, slots, period=None):
    """Generalised diagonal i of M (n_out x n_in) for output period d and an
    input that repeats every `period` slots (default: slots): entry j is
    M[j mod d][(j+i) mod period] when both indices are in range."""
    period = slots if period is None else period
    n_out, n_in = M.shape
    j = np.arange(slots)
    r = j % d
    c = (j + i) % period
    v = np.zeros(slots)
    ok = (r < n_out) & (c < n_in)
    v[ok] = M[r[ok], c[ok]]
    return v


def bsgs_split(d):
    b1 = 1 << ((clog2(d) + 1) // 2)
    return b1, d // b1


def matvec_partial(ev, x, M, d, t, S=1, period=None, shared_moddown=False):
    """z = sum_{i<d} diag_{iS} * rot(x, iS) at level t by baby-step giant-step:
    z = sum_gi rot( sum_bi rot(diag_{(gi b1 + bi) S}, -gi b1 S) * rot(x, bi S), gi b1 S ),
    diagonals of M taken with output period d S (for S = 1 every diagonal i < d;
    for M = W (x) I_S the others are zero).  x is mod-dropped to t+1 before
    the baby-step rotations.  If x repeats every `period` slots, so do the
    diagonals, and z needs folding within one period only.  shared_moddown:
    the giant-step rotations share one ModDown (ev.rotate_sum)."""
    slots = ev.ctx.p.slots
    b1, g1 = bsgs_split(d)
    D = d * S
    xd = ev.mod_drop(x, t + 1)
    rots = [xd] + [ev.rotate(xd, bi * S) for bi in range(1, b1)]
    z = None
    items = []
    for gi in range(g1):
        terms = []
        for bi in range(b1):
            dv = np.roll(diag_vector(M, D, (gi * b1 + bi) * S, slots, period), gi * b1 * S)
            terms.append((rots[bi], dv))
        inner = ev.lincomb(terms, t)
        if shared_moddown:
            items.append((inner, gi * b1 * S))
            continue
        if gi:
            inner = ev.rotate(inner, gi * b1 * S)
        z = inner if z is None else ev.add(z, inner)
    return ev.rotate_sum(items) if shared_moddown else z


def fold(ev, z, d, period=None):
    """z <- z + rot(z, s) for s = period/2, period/4, ..., d (d: the output
    period; period: the period of z, default slots)."""
    s = (ev.ctx.p.slots if period is None else period) // 2
    while s >= d:
        z = ev.add(z, ev.rotate(z, s))
        s //= 2
    return z


def permutation_offsets(L, n_blk, S, slots):
    """The homomorphic permutation of the naive method (Algorithm 3's P applied
    to the ciphertext): slot (i (g+k) + m) S + s receives slot
    m n_blk + i S + s (basis m of input i of vector s).  Returns the signed
    offset src - dst of every destination (in (-slots/2, slots/2]) and the
    baby-step width b1 = the power of two >= sqrt(2 R + 1), R the largest
    |offset|; offset o = g b1 + b splits into giant g (floor) and baby
    b in [0, b1)."""
    nb = L.g + L.k
    dst, off = [], []
    for i in range(L.n_in):
        for m in range(nb):
            for s in range(S):
                d = (i * nb + m) * S + s
                o = (m * n_blk + i * S + s - d) % slots
                if o > slots // 2:
                    o -= slots
                dst.append(d)
                off.append(o)
    R = max(abs(o) for o in off)
    b1 = pow2ceil(int(math.ceil(math.sqrt(2 * R + 1))))
    return np.array(dst), np.array(off), b1


def permute(ev, x, L, n_blk, S, t):
    """z[d] = x[src(d)] for the naive method's permutation, zero elsewhere, at
    level t, by the diagonal method with baby-step giant-step rotations:
    z = sum_g rot( sum_b rot(diag_(g b1 + b), -g b1) * rot(x, b), g b1 ),
    diag_o the 0/1 vector of the destinations with offset o (one ct x pt
    product per non-zero diagonal)."""
    slots = ev.ctx.p.slots
    dst, off, b1 = permutation_offsets(L, n_blk, S, slots)
    giants = sorted(set(int(o) // b1 for o in off))
    babies = sorted(set(int(o) - (int(o) // b1) * b1 for o in off))
    xd = ev.mod_drop(x, t + 1)
    rots = {b: (xd if b == 0 else ev.rotate(xd, b)) for b in babies}
    z = None
    for g in giants:
        terms = []
        for b in babies:
            sel = dst[off == g * b1 + b]
            if len(sel) == 0:
                continue
            dv = np.zeros(slots)
            dv[sel] = 1.0
            terms.append((rots[b], np.roll(dv, g * b1)))
        inner = ev.lincomb(terms, t)
        if g:
            inner = ev.rotate(inner, g * b1)
        z = inner if z is None else ev.add(z, inner)
    return z


def chunk_bounds(L, slots, S=1):
    """Feature ranges [b_c, b_{c+1}) of the first layer's input ciphertexts:
    each chunk holds as many consecutive features as its repeat-packed
    footprint (chunk size times S times 2^ceil(log2(g+2k))) allows in the
    slots, the last one the rest."""
    cap = (slots >> clog2(L.g + 2 * L.k)) // S
    if cap < 1:
        raise ValueError("g+2k copies of one input exceed the slots")
    return list(range(0, L.n_in, cap)) + [L.n_in]


def pack_samples(X, S):
    """Slot vector of S input vectors X (S x n): feature i of vector s in slot i S + s."""
    X = np.atleast_2d(np.asarray(X, np.float64))
    assert X.shape[0] == S
    return X.T.reshape(-1)


def strided(M, S, col_blocks=1, n_blk=None):
    """W (x) I_S in the slot layout: M (n_out x col_blocks n_w, block m of
    width n_w) -> rows o S + s, columns m n_blk + i S + s (n_blk >= n_w S)."""
    n_out, cols = M.shape
    n_w = cols // col_blocks
    n_blk = n_w * S if n_blk is None else n_blk
    out = np.zeros((n_out * S, col_blocks * n_blk))
    for m in range(col_blocks):
        for s in range(S):
            out[s::S, m * n_blk + s:m * n_blk + n_w * S:S] = M[:, m * n_w:(m + 1) * n_w]
    return out


def sub_layer(L, lo, hi):
    """The layer restricted to input features [lo, hi)."""
    return dataclasses.replace(L, n_in=hi - lo, wb=L.wb[:, lo:hi], ws=L.ws[:, lo:hi], c=L.c[:, lo:hi])


def shared_comparison(L, n_blk, first, slots):
    """Whether the repeat-packed input holds g+2k+1 blocks (the first layer's
    2^ceil(log2(g+2k)) copies, or a periodic hidden input), so that
    bspline_basis can share one comparison between both of its inputs."""
    r = L.g + 2 * L.k + 1
    blocks = (1 << clog2(L.g + 2 * L.k)) if first else slots // n_blk
    return blocks >= r and r * n_blk <= slots


def hidden_period(L, n_blk, slots, circ=RESTRUCTURED):
    """The period of a hidden layer's block layout.  Its input repeats every
    n_blk slots, so with folded_period the layout (g+2k blocks of
    comparisons, or g+2k+1 when the second comparison is shared; g+k bases
    and, fused, the masked SiLU block) repeats every P = next power of two of
    that many slots, the products repeat every P as well and the fold runs
    over one period.  Otherwise P is all the slots."""
    if not circ.folded_period:
        return slots
    r = L.g + 2 * L.k + 1
    nblocks = r if (circ.shared_comparison or (circ.fused_linear and L.k == 0)) else r - 1
    return min(slots, pow2ceil(nblocks * n_blk))


def layer_part(ev, x, L, n_blk, first, d, S=1, circ=PAPER):
    """Both branches of one layer on one input ciphertext, before the fold.
    n_blk: slots per input block (n_in S for a first layer).  Returns the
    pre-fold products: [z] for fused_linear (the SiLU branch evaluated on the
    repeat-packed input with its coefficients masked to block g+k, the first
    block the g+k bases leave free, added to the bases, and one product with
    [W_f | W_b], g+k+1 column blocks), else [z_f, z_b] (W_f times the bases,
    W_b times the SiLU values of x), both landing at the same level."""
    slots = ev.ctx.p.slots
    nb = L.g + L.k
    width = L.n_in * S
    if circ.naive_permutation and (circ.fused_linear or circ.folded_period):
        raise ValueError("the naive permutation excludes the fused linear layers and the folded period")
    period = slots if first else hidden_period(L, n_blk, slots, circ)
    xr = repeat_pack(ev, x, n_blk, clog2(L.g + 2 * L.k)) if first else x
    shared = circ.shared_comparison and shared_comparison(L, n_blk, first, slots)
    b = bspline_basis(ev, xr, L, n_blk, width, shared, period)
    if circ.fused_linear:
        mask = np.zeros(period)
        mask[nb * n_blk:nb * n_blk + width] = 1.0
        s = cheb_eval(ev, xr, L.silu_coeffs, L.silu_lo, L.silu_hi, np.tile(mask, slots // period))
        t = min(b.level, s.level) - 1
        z = ev.add(ev.mod_drop(b, t + 1), ev.mod_drop(s, t + 1))
        W = strided(np.hstack([fused_weights(L, L.n_in), L.wb]), S, nb + 1, n_blk)
        return [matvec_partial(ev, z, W, d, t, S, period, circ.shared_moddown)]
    s = cheb_eval(ev, x, L.silu_coeffs, L.silu_lo, L.silu_hi)
    Wb = strided(L.wb, S, 1, n_blk)
    if circ.naive_permutation:
        # no lazy combination: the bases permuted into row order, then W'
        bp = permute(ev, b, L, n_blk, S, b.level - 1)
        t = min(bp.level, s.level) - 1
        Wr = strided(lazy_weights(L), S, 1, L.n_in * nb * S)
        return [matvec_partial(ev, bp, Wr, d, t, S, period, circ.shared_moddown),
                matvec_partial(ev, s, Wb, d, t, S, period, circ.shared_moddown)]
    t = min(b.level, s.level) - 1
    Wf = strided(fused_weights(L, L.n_in), S, nb, n_blk)
    return [matvec_partial(ev, b, Wf, d, t, S, period, circ.shared_moddown),
            matvec_partial(ev, s, Wb, d, t, S, period, circ.shared_moddown)]


def layer_forward(ev, xs, L, n_blk, first, S=1, circ=PAPER):
    """xs: the first layer's chunk ciphertexts (see chunk_bounds), else [x];
    n_blk: the previous output period (later layers).  Returns the output and
    its period d S.  The chunks' pre-fold products are added (per linear
    layer), then each sum is folded; without fused_linear the layer output is
    fold(z_f) + fold(z_b)."""
    d = pow2ceil(L.n_out)
    if first:
        bounds = chunk_bounds(L, ev.ctx.p.slots, S)
        parts = [(sub_layer(L, lo, hi), (hi - lo) * S) for lo, hi in zip(bounds[:-1], bounds[1:])]
    else:
        parts = [(L, n_blk)]
    if len(xs) != len(parts):
        raise ValueError("layer takes %d input ciphertexts, got %d" % (len(parts), len(xs)))
    zs = None
    for x, (Lc, nb) in zip(xs, parts):
        zc = layer_part(ev, x, Lc, nb, first, d, S, circ)
        zs = zc if zs is None else [ev.add(a, b) for a, b in zip(zs, zc)]
    period = ev.ctx.p.slots if first else hidden_period(L, n_blk, ev.ctx.p.slots, circ)
    y = fold(ev, zs[0], d * S, period)
    for z in zs[1:]:
        y = ev.add(y, fold(ev, z, d * S, period))
    return y, d * S


def eval_kan(ev, ct, layers, refresh=None, S=1, circ=PAPER):
    """Run the layers on ct: one ciphertext (input in slots [0, n_in S)) or the
    list of the first layer's chunk ciphertexts (chunk c holds features
    [b_c, b_{c+1}) in slots [0, (b_{c+1} - b_c) S)); with S vectors per
    ciphertext, feature i of vector s is in slot i S + s, and output o of
    vector s comes out in slot o S + s.  `refresh`, if given, is called
    between layers with the ciphertext and returns a fresh one at the top
    level (the client-aided stand-in for bootstrapping).  `circ` selects the
    restructurings (default: the paper's order)."""
    xs = list(ct) if isinstance(ct, (list, tuple)) else [ct]
    n_blk = 0
    for li, L in enumerate(layers):
        if li > 0 and refresh is not None:
            xs = [refresh(xs[0], li)]
        x, n_blk = layer_forward(ev, xs, L, n_blk, li == 0, S, circ)
        xs = [x]
    return xs[0]


def rotation_steps(layers, slots, S=1, circ=PAPER):
    """Every rotation amount the circuit uses (for key generation)."""
    steps = set()
    n_blk = 0
    for li, L in enumerate(layers):
        d = pow2ceil(L.n_out)
        if li == 0:
            bounds = chunk_bounds(L, slots, S)
            for nb in set((hi - lo) * S for lo, hi in zip(bounds[:-1], bounds[1:])):
                for j in range(1, clog2(L.g + 2 * L.k) + 1):
                    steps.add(-nb * (1 << (j - 1)))
                steps.add(nb)
        else:
            steps.add(n_blk)
        if circ.naive_permutation:
            parts = ([(sub_layer(L, lo, hi), (hi - lo) * S) for lo, hi in
                      zip(chunk_bounds(L, slots, S)[:-1], chunk_bounds(L, slots, S)[1:])] if li == 0
                     else [(L, n_blk)])
            for Lc, nbk in parts:
                _, off, pb1 = permutation_offsets(Lc, nbk, S, slots)
                for o in set(int(v) for v in off):
                    g, b = o // pb1, o - (o // pb1) * pb1
                    if b:
                        steps.add(b)
                    if g:
                        steps.add(g * pb1)
        b1, g1 = bsgs_split(d)
        steps.update(bi * S for bi in range(1, b1))
        steps.update(gi * b1 * S for gi in range(1, g1))
        s = (slots if li == 0 else hidden_period(L, n_blk, slots, circ)) // 2
        while s >= d * S:
            steps.add(s)
            s //= 2
        n_blk = d * S
    return sorted(steps)
