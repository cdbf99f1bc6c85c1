"""Plain CPU RNS-CKKS reference (the oracle), Python layer over ckks_oracle.c.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.

Follows the paper's Preliminaries ("Homomorphic Encryption": SIMD ciphertext
addition, subtraction, multiplication and rotation under RNS-CKKS; rotation by
t > 0 moves slots left).  Ciphertexts are kept in coefficient form with one
row of N residues per RNS limb.  Every ciphertext at level l carries the
canonical scale S[l] of that level (S[L] = 2^scale_bits,
S[l-1] = S[l]*S[l]/q_l), so scale bookkeeping is a function of the level only.
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force=False):
    """Compile ckks_oracle.c with gcc into liboracle.so (next to the source)."""
    src = os.path.join(_HERE, "ckks_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-fopenmp", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, i32, d, u32 = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_uint32
        sig = {
            "oc_powm": (u64, [u64, u64, u64]),
            "oc_invm": (u64, [u64, u64]),
            "oc_is_prime": (i32, [u64]),
            "oc_gen_primes": (i32, [i32, i32, i32, i32, i32, i32, i32, i32, _u64p, _u64p, _dp]),
            "oc_find_psi": (u64, [u64, i32]),
            "oc_ntt_fwd": (None, [_u64p, i32, u64]),
            "oc_ntt_inv": (None, [_u64p, i32, u64]),
            "oc_negacyclic_mul": (None, [_u64p, _u64p, _u64p, i32, u64]),
            "oc_schoolbook_mul": (None, [_u64p, _u64p, _u64p, i32, u64]),
            "oc_poly_add": (None, [_u64p, _u64p, _u64p, i32, i32, _u64p]),
            "oc_poly_sub": (None, [_u64p, _u64p, _u64p, i32, i32, _u64p]),
            "oc_poly_mul": (None, [_u64p, _u64p, _u64p, i32, i32, _u64p]),
            "oc_poly_mul_scalar": (None, [_u64p, _u64p, _u64p, i32, i32, _u64p]),
            "oc_automorph": (None, [_u64p, _u64p, i32, i32, _u64p, u64]),
            "oc_rescale": (None, [_u64p, _u64p, i32, i32, _u64p]),
            "oc_bconv": (None, [_u64p, i32, _u64p, _u64p, i32, _u64p, i32]),
            "oc_moddown": (None, [_u64p, _u64p, i32, i32, i32, _u64p, _u64p]),
            "oc_keyswitch": (None, [_u64p, i32, _u64p, i32, i32, i32, _u64p, _u64p, i32, u64, _u64p, _u64p]),
            "oc_keyswitch_acc": (None, [_u64p, i32, _u64p, i32, i32, i32, _u64p, _u64p, i32, u64, _u64p, _u64p]),
            "oc_chacha20_block": (None, [_u32p, u32, _u32p, _u32p]),
            "oc_sample_uniform": (None, [u64, u32, u32, u32, u64, i32, _u64p]),
            "oc_sample_ternary": (None, [u64, u32, u32, u32, i32, _i64p]),
            "oc_sample_sparse_ternary": (None, [u64, u32, u32, u32, i32, i32, _i64p]),
            "oc_sample_gauss": (None, [u64, u32, u32, u32, d, i32, _i64p]),
            "oc_gauss_table": (None, [d, _u64p]),
            "oc_small_to_rns": (None, [_i64p, _u64p, i32, i32, _u64p]),
            "oc_gen_switch_key": (None, [u64, u32, _u64p, _u64p, i32, i32, i32, _u64p, _u64p, i32, d, _u64p]),
            "oc_encode": (None, [_dp, i32, d, i32, _u64p, i32, _u64p]),
            "oc_encode_c": (None, [_dp, _dp, i32, d, i32, _u64p, i32, _u64p]),
            "oc_decode_c": (None, [_u64p, u64, d, i32, i32, _dp, _dp]),
            "oc_root_table": (None, [i32, _dp, _dp]),
            "oc_encode_coeff_direct_c": (d, [_dp, _dp, i32, d, i32, u64]),
            "oc_encode_const": (None, [d, d, _u64p, i32, _u64p]),
            "oc_encode_coeffs_dd": (None, [_dp, i32, d, i32, _dp, _dp]),
            "oc_decode": (None, [_u64p, u64, d, i32, i32, _dp]),
            "oc_encode_coeff_direct": (d, [_dp, i32, d, i32, u64]),
            "oc_set_threads": (None, [i32]),
            "oc_get_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def set_threads(n):
    """Host threads for the oracle's limb loops (n <= 0: all cores); results do
    not depend on it."""
    lib().oc_set_threads(int(n))


def get_threads():
    return int(lib().oc_get_threads())


def P(a):
    """ctypes pointer to a contiguous numpy array."""
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.uint64:
        return a.ctypes.data_as(_u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_i64p)
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.uint32:
        return a.ctypes.data_as(_u32p)
    raise TypeError(a.dtype)


def u64a(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Params:
    """RNS-CKKS parameter set: ring degree 2^logN, base prime bits, L scale
    primes of scale_bits, alpha special primes, key-switch digits of `w`
    consecutive Q limbs, Gaussian sigma.  boot_levels > 0 makes the top
    boot_levels primes (the levels a bootstrapping consumes) boot_bits wide,
    with canonical scales near 2^boot_bits there; h > 0 draws a sparse
    ternary secret with exactly h non-zero coefficients (uniform ternary
    otherwise)."""
    logN: int
    L: int
    scale_bits: int
    alpha: int
    w: int
    base_bits: int = 60
    special_bits: int = 60
    sigma: float = 3.2
    boot_levels: int = 0
    boot_bits: int = 0
    h: int = 0

    @property
    def N(self):
        return 1 << self.logN

    @property
    def slots(self):
        return self.N // 2

    @property
    def top_level(self):
        """the top computation level (fresh encryptions and bootstrapping
        results start here)"""
        return self.L - self.boot_levels


# rotation "step" naming the complex conjugation (Galois element 2N - 1)
STEP_CONJUGATE = -(1 << 31)


class Context:
    """Prime chain, canonical per-level scales and the Galois helpers."""

    def __init__(self, params: Params):
        self.p = params
        L = lib()
        q = np.zeros(params.L + 1, np.uint64)
        pp = np.zeros(params.alpha, np.uint64)
        S = np.zeros(params.L + 1, np.float64)
        L.oc_gen_primes(params.logN, params.base_bits, params.L, params.scale_bits, params.alpha,
                        params.special_bits, params.boot_levels, params.boot_bits, P(q), P(pp), P(S))
        self.q = q
        self.pm = pp
        self.S = S
        self.all_mods = u64a(list(q) + list(pp))

    def galois_elt(self, t):
        """Galois element 5^t mod 2N for a left rotation by t slots
        (2N - 1, the complex conjugation, for STEP_CONJUGATE)."""
        N = self.p.N
        if t == STEP_CONJUGATE:
            return 2 * N - 1
        t %= N // 2
        return pow(5, t, 2 * N)

    def mods(self, l):
        return u64a(self.q[: l + 1])


# --------------------------------------------------------------------------
# keys and ciphertexts
# --------------------------------------------------------------------------
@dataclass
class Ciphertext:
    level: int
    c0: np.ndarray  # (level+1, N) uint64, coefficient form
    c1: np.ndarray


class Keys:
    """Secret key (client side) and switching keys, all in coefficient form."""

    def __init__(self, ctx: Context, seed: int, rot_steps):
        self.ctx = ctx
        p = ctx.p
        N = p.N
        L = lib()
        s = np.zeros(N, np.int64)
        if p.h > 0:
            L.oc_sample_sparse_ternary(seed, 1, 0, 0, p.logN, p.h, P(s))
        else:
            L.oc_sample_ternary(seed, 1, 0, 0, p.logN, P(s))
        self.s_small = s
        ktot = p.L + 1 + p.alpha
        self.s_res = np.zeros((ktot, N), np.uint64)
        L.oc_small_to_rns(P(s), P(self.s_res), ktot, p.logN, P(ctx.all_mods))
        self.keys = {}
        dnum = (p.L + 1 + p.w - 1) // p.w
        # relinearisation key: s' = s^2
        s2 = np.zeros_like(self.s_res)
        L.oc_poly_mul(P(self.s_res), P(self.s_res), P(s2), ktot, p.logN, P(ctx.all_mods))
        self.keys[0] = self._gen(seed, 0, s2, dnum)
        # Galois keys: s' = sigma_g(s)
        for t in sorted(set(rot_steps)):
            g = ctx.galois_elt(t)
            if g == 1 or g in self.keys:
                continue
            sg = np.zeros_like(self.s_res)
            L.oc_automorph(P(self.s_res), P(sg), ktot, p.logN, P(ctx.all_mods), g)
            self.keys[g] = self._gen(seed, g, sg, dnum)

    def _gen(self, seed, key_id, sp, dnum):
        p = self.ctx.p
        ktot = p.L + 1 + p.alpha
        out = np.zeros((dnum, 2, ktot, p.N), np.uint64)
        lib().oc_gen_switch_key(seed, key_id, P(self.s_res), P(sp), p.L, p.alpha, p.w, P(self.ctx.q),
                                P(self.ctx.pm), p.logN, p.sigma, P(out))
        return out


class Oracle:
    """RNS-CKKS evaluator over a Context and Keys.  The operations mirror the
    paper's homomorphic primitives; the helpers `lincomb`, `level_down` and
    `tensor`/`relin_rescale` fix how constants are encoded and where rescales
    happen, so that two independent implementations of the same circuit reach
    identical residues."""

    def __init__(self, ctx: Context, keys: Keys = None):
        self.ctx = ctx
        self.keys = keys
        self.lib = lib()
        self.count = {"ks": 0, "rescale": 0}

    # -- encoding ----------------------------------------------------------
    def encode(self, z, scale, nl):
        """round(scale tau^-1(z)) over nl limbs; z real or complex"""
        p = self.ctx.p
        out = np.zeros((nl, p.N), np.uint64)
        if np.iscomplexobj(z):
            re = np.ascontiguousarray(np.real(z), np.float64)
            im = np.ascontiguousarray(np.imag(z), np.float64)
            self.lib.oc_encode_c(P(re), P(im), len(re), scale, p.logN, P(self.ctx.all_mods[:nl].copy()), nl,
                                 P(out))
            return out
        z = np.ascontiguousarray(np.asarray(z, np.float64))
        self.lib.oc_encode(P(z), len(z), scale, p.logN, P(self.ctx.all_mods[:nl].copy()), nl, P(out))
        return out

    def encode_const(self, c, scale, nl):
        out = np.zeros(nl, np.uint64)
        self.lib.oc_encode_const(float(c), scale, P(self.ctx.all_mods[:nl].copy()), nl, P(out))
        return out

    def decode_c(self, c_limb0, scale, nz):
        """complex slots of a centred limb-0 polynomial"""
        p = self.ctx.p
        re = np.zeros(nz, np.float64)
        im = np.zeros(nz, np.float64)
        self.lib.oc_decode_c(P(np.ascontiguousarray(c_limb0)), int(self.ctx.q[0]), scale, p.logN, nz, P(re), P(im))
        return re + 1j * im

    def decode(self, c_limb0, scale, nz):
        p = self.ctx.p
        z = np.zeros(nz, np.float64)
        self.lib.oc_decode(P(np.ascontiguousarray(c_limb0)), int(self.ctx.q[0]), scale, p.logN, nz, P(z))
        return z

    # -- client side ----------------------------------------------------------
    def encrypt(self, z, seed, level=None):
        """Secret-key encryption (-a*s + e + m, a) at the top computation level
        (the client holds s, as in the paper's threat model)."""
        ctx, p = self.ctx, self.ctx.p
        l = p.top_level if level is None else level
        nl = l + 1
        m = self.encode(z, ctx.S[l], nl)
        a = np.zeros((nl, p.N), np.uint64)
        for t in range(nl):
            self.lib.oc_sample_uniform(seed, 4, 0, t, int(ctx.q[t]), p.logN, P(a[t]))
        e = np.zeros(p.N, np.int64)
        self.lib.oc_sample_gauss(seed, 5, 0, 0, p.sigma, p.logN, P(e))
        er = np.zeros((nl, p.N), np.uint64)
        mods = ctx.mods(l)
        self.lib.oc_small_to_rns(P(e), P(er), nl, p.logN, P(mods))
        s = np.ascontiguousarray(self.keys.s_res[:nl])
        as_ = np.zeros_like(a)
        self.lib.oc_poly_mul(P(a), P(s), P(as_), nl, p.logN, P(mods))
        c0 = np.zeros_like(a)
        self.lib.oc_poly_sub(P(er), P(as_), P(c0), nl, p.logN, P(mods))
        self.lib.oc_poly_add(P(c0), P(m), P(c0), nl, p.logN, P(mods))
        return Ciphertext(l, c0, a)

    def phase(self, ct):
        """c0 + c1*s on limb q0, coefficient form"""
        p = self.ctx.p
        q0 = u64a([self.ctx.q[0]])
        m = np.zeros((1, p.N), np.uint64)
        self.lib.oc_poly_mul(P(np.ascontiguousarray(ct.c1[:1])), P(np.ascontiguousarray(self.keys.s_res[:1])),
                             P(m), 1, p.logN, P(q0))
        self.lib.oc_poly_add(P(m), P(np.ascontiguousarray(ct.c0[:1])), P(m), 1, p.logN, P(q0))
        return m[0]

    def decrypt_c(self, ct, nz):
        """complex slots of the decryption"""
        return self.decode_c(self.phase(ct), self.ctx.S[ct.level], nz)

    def decrypt(self, ct, nz):
        """m = c0 + c1*s on limb q0 (|m| < q0/2), then decode at S[level]."""
        p = self.ctx.p
        q0 = u64a([self.ctx.q[0]])
        c0 = np.ascontiguousarray(ct.c0[:1])
        c1 = np.ascontiguousarray(ct.c1[:1])
        s = np.ascontiguousarray(self.keys.s_res[:1])
        m = np.zeros((1, p.N), np.uint64)
        self.lib.oc_poly_mul(P(c1), P(s), P(m), 1, p.logN, P(q0))
        self.lib.oc_poly_add(P(m), P(c0), P(m), 1, p.logN, P(q0))
        return self.decode(m[0], self.ctx.S[ct.level], nz)

    # -- level-preserving ops -------------------------------------------------
    def _binop(self, fn, a, b, nl):
        p = self.ctx.p
        out = np.zeros((nl, p.N), np.uint64)
        fn(P(np.ascontiguousarray(a[:nl])), P(np.ascontiguousarray(b[:nl])), P(out), nl, p.logN,
           P(self.ctx.mods(nl - 1)))
        return out

    def add(self, a, b):
        assert a.level == b.level, (a.level, b.level)
        nl = a.level + 1
        f = self.lib.oc_poly_add
        return Ciphertext(a.level, self._binop(f, a.c0, b.c0, nl), self._binop(f, a.c1, b.c1, nl))

    def sub(self, a, b):
        assert a.level == b.level
        nl = a.level + 1
        f = self.lib.oc_poly_sub
        return Ciphertext(a.level, self._binop(f, a.c0, b.c0, nl), self._binop(f, a.c1, b.c1, nl))

    def mul_int(self, a, k):
        """multiply by a small signed integer (exact, scale unchanged)."""
        mods = self.ctx.mods(a.level)
        res = u64a([(k % int(m)) for m in mods])
        nl = a.level + 1
        p = self.ctx.p
        outs = []
        for c in (a.c0, a.c1):
            o = np.zeros((nl, p.N), np.uint64)
            self.lib.oc_poly_mul_scalar(P(np.ascontiguousarray(c)), P(res), P(o), nl, p.logN, P(mods))
            outs.append(o)
        return Ciphertext(a.level, outs[0], outs[1])

    def add_const(self, a, c):
        """add the constant c encoded at the ciphertext's scale."""
        nl = a.level + 1
        r = self.encode_const(c, self.ctx.S[a.level], nl)
        c0 = a.c0.copy()
        mods = self.ctx.mods(a.level)
        for t in range(nl):
            c0[t, 0] = (int(c0[t, 0]) + int(r[t])) % int(mods[t])
        return Ciphertext(a.level, c0, a.c1.copy())

    def add_vec(self, a, z):
        """add the slot vector z encoded at the ciphertext's scale."""
        nl = a.level + 1
        m = self.encode(z, self.ctx.S[a.level], nl)
        return Ciphertext(a.level, self._binop(self.lib.oc_poly_add, a.c0, m, nl), a.c1.copy())

    def mul_i(self, a):
        """multiply by the monomial X^(N/2): every slot times i (zeta^(5^j N/2)
        = i because 5^j = 1 mod 4); a negacyclic shift, exact"""
        N = self.ctx.p.N
        h = N // 2
        mods = self.ctx.mods(a.level)[:, None]
        outs = []
        for c in (a.c0, a.c1):
            o = np.empty_like(c)
            o[:, h:] = c[:, :h]
            lo = c[:, h:]
            o[:, :h] = np.where(lo == 0, np.uint64(0), mods - lo)
            outs.append(o)
        return Ciphertext(a.level, outs[0], outs[1])

    def mod_raise(self, a):
        """ModRaise: the residues mod q_0 of a level-0 ciphertext, read as
        centred integers in (-q_0/2, q_0/2), lifted to every prime of the top
        level L (the plaintext becomes m + q_0 I for a small integer
        polynomial I)"""
        assert a.level == 0
        p = self.ctx.p
        q0 = int(self.ctx.q[0])
        mods = self.ctx.mods(p.L)
        outs = []
        for c in (a.c0, a.c1):
            v = c[0].astype(np.int64)
            v = np.where(2 * c[0] > np.uint64(q0), v - np.int64(q0), v)
            o = np.zeros((p.L + 1, p.N), np.uint64)
            self.lib.oc_small_to_rns(P(np.ascontiguousarray(v)), P(o), p.L + 1, p.logN, P(mods))
            outs.append(o)
        return Ciphertext(p.L, outs[0], outs[1])

    def mod_drop(self, a, l):
        assert l <= a.level
        return Ciphertext(l, a.c0[: l + 1].copy(), a.c1[: l + 1].copy())

    # -- rescale and key switching ---------------------------------------------
    def _rescale_poly(self, c, l):
        p = self.ctx.p
        out = np.zeros((l, p.N), np.uint64)
        self.lib.oc_rescale(P(np.ascontiguousarray(c[: l + 1])), P(out), l, p.logN, P(self.ctx.q))
        return out

    def rescale(self, a):
        self.count["rescale"] += 1
        l = a.level
        return Ciphertext(l - 1, self._rescale_poly(a.c0, l), self._rescale_poly(a.c1, l))

    def keyswitch(self, d, l, key_id, galois=0):
        p = self.ctx.p
        self.count["ks"] += 1
        u0 = np.zeros((l + 1, p.N), np.uint64)
        u1 = np.zeros((l + 1, p.N), np.uint64)
        key = self.keys.keys[key_id]
        self.lib.oc_keyswitch(P(np.ascontiguousarray(d[: l + 1])), l, P(key), p.L, p.alpha, p.w, P(self.ctx.q),
                              P(self.ctx.pm), p.logN, galois, P(u0), P(u1))
        return u0, u1

    def tensor(self, a, b):
        """(d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) at the common level."""
        assert a.level == b.level, (a.level, b.level)
        nl = a.level + 1
        f = self.lib.oc_poly_mul
        d0 = self._binop(f, a.c0, b.c0, nl)
        d1 = self._binop(self.lib.oc_poly_add, self._binop(f, a.c0, b.c1, nl), self._binop(f, a.c1, b.c0, nl), nl)
        d2 = self._binop(f, a.c1, b.c1, nl)
        return [a.level, d0, d1, d2]

    def tensor_add(self, t1, t2):
        assert t1[0] == t2[0]
        nl = t1[0] + 1
        f = self.lib.oc_poly_add
        return [t1[0]] + [self._binop(f, x, y, nl) for x, y in zip(t1[1:], t2[1:])]

    def relin_rescale(self, t):
        """relinearise d2 with the key for s^2, then rescale."""
        l, d0, d1, d2 = t
        u0, u1 = self.keyswitch(d2, l, 0)
        nl = l + 1
        f = self.lib.oc_poly_add
        c = Ciphertext(l, self._binop(f, d0, u0, nl), self._binop(f, d1, u1, nl))
        return self.rescale(c)

    def mul(self, a, b):
        """ct x ct: tensor, relinearise, rescale (level l -> l-1)."""
        return self.relin_rescale(self.tensor(a, b))

    def rotate(self, a, t):
        """rot(a, t): slots move left by t (right for t < 0)."""
        g = self.ctx.galois_elt(t)
        if g == 1:
            return a
        p = self.ctx.p
        l = a.level
        nl = l + 1
        u0, u1 = self.keyswitch(a.c1, l, g, galois=g)
        s0 = np.zeros((nl, p.N), np.uint64)
        mods = self.ctx.mods(l)
        self.lib.oc_automorph(P(np.ascontiguousarray(a.c0[:nl])), P(s0), nl, p.logN, P(mods), g)
        return Ciphertext(l, self._binop(self.lib.oc_poly_add, s0, u0, nl), u1)

    def rotate_sum(self, items):
        """sum_i rot(x_i, t_i) for (x_i, t_i) in items, all at one level, with
        a single ModDown: each rotation's key-switch accumulators (over
        Q_l u P, before ModDown, the automorphism applied to the extended
        digits as in rotate) are added up and divided by P once, and the
        rotated c_0 parts and the unrotated terms are added in Q_l (the
        ModDown hoisted out of a sum of rotations, Bossuat, Mouchet,
        Troncoso-Pastoriza and Hubaux 2021).  Equal to the sum of the
        separate rotations up to the rounding of the divisions by P."""
        p = self.ctx.p
        l = items[0][0].level
        nl, next_ = l + 1, l + 1 + p.alpha
        mods_q = self.ctx.mods(l)
        mods_qp = u64a(list(self.ctx.q[:nl]) + list(self.ctx.pm))
        add = self.lib.oc_poly_add
        b0 = np.zeros((nl, p.N), np.uint64)
        b1 = np.zeros((nl, p.N), np.uint64)
        a0 = np.zeros((next_, p.N), np.uint64)
        a1 = np.zeros((next_, p.N), np.uint64)
        rotated = False
        for x, t in items:
            assert x.level == l, (x.level, l)
            g = self.ctx.galois_elt(t)
            if g == 1:
                add(P(b0), P(np.ascontiguousarray(x.c0[:nl])), P(b0), nl, p.logN, P(mods_q))
                add(P(b1), P(np.ascontiguousarray(x.c1[:nl])), P(b1), nl, p.logN, P(mods_q))
                continue
            self.count["ks"] += 1
            u0 = np.zeros((next_, p.N), np.uint64)
            u1 = np.zeros((next_, p.N), np.uint64)
            self.lib.oc_keyswitch_acc(P(np.ascontiguousarray(x.c1[:nl])), l, P(self.keys.keys[g]), p.L, p.alpha,
                                      p.w, P(self.ctx.q), P(self.ctx.pm), p.logN, g, P(u0), P(u1))
            add(P(a0), P(u0), P(a0), next_, p.logN, P(mods_qp))
            add(P(a1), P(u1), P(a1), next_, p.logN, P(mods_qp))
            s0 = np.zeros((nl, p.N), np.uint64)
            self.lib.oc_automorph(P(np.ascontiguousarray(x.c0[:nl])), P(s0), nl, p.logN, P(mods_q), g)
            add(P(b0), P(s0), P(b0), nl, p.logN, P(mods_q))
            rotated = True
        if rotated:
            for a, b in ((a0, b0), (a1, b1)):
                u = np.zeros((nl, p.N), np.uint64)
                self.lib.oc_moddown(P(a), P(u), nl, p.alpha, p.logN, P(self.ctx.q), P(self.ctx.pm))
                add(P(b), P(u), P(b), nl, p.logN, P(mods_q))
        return Ciphertext(l, b0, b1)

    # -- plaintext products with a target level ------------------------------
    def lincomb(self, terms, t):
        """sum_i ct_i * z_i, landing exactly at level t with scale S[t].

        Every ct_i (level l_i >= t+1) is mod-dropped to t+1 and multiplied by
        z_i (a constant or a slot vector) encoded at
        X_i = (S[t] * q_{t+1}) / S[l_i]; the products are summed and rescaled
        once by q_{t+1}."""
        ctx, p = self.ctx, self.ctx.p
        nl = t + 2
        mods = ctx.mods(t + 1)
        acc0 = np.zeros((nl, p.N), np.uint64)
        acc1 = np.zeros((nl, p.N), np.uint64)
        for ct, z in terms:
            assert ct.level >= t + 1, (ct.level, t)
            X = ctx.S[t] * float(ctx.q[t + 1]) / ctx.S[ct.level]
            c0 = np.ascontiguousarray(ct.c0[:nl])
            c1 = np.ascontiguousarray(ct.c1[:nl])
            if np.isscalar(z):
                r = self.encode_const(z, X, nl)
                f = self.lib.oc_poly_mul_scalar
                m0 = np.zeros_like(acc0)
                m1 = np.zeros_like(acc1)
                f(P(c0), P(r), P(m0), nl, p.logN, P(mods))
                f(P(c1), P(r), P(m1), nl, p.logN, P(mods))
            else:
                pt = self.encode(z, X, nl)
                m0 = self._binop(self.lib.oc_poly_mul, c0, pt, nl)
                m1 = self._binop(self.lib.oc_poly_mul, c1, pt, nl)
            acc0 = self._binop(self.lib.oc_poly_add, acc0, m0, nl)
            acc1 = self._binop(self.lib.oc_poly_add, acc1, m1, nl)
        return self.rescale(Ciphertext(t + 1, acc0, acc1))

    def level_down(self, a, t):
        """bring a to level t (< a.level) with scale S[t]: multiply by 1."""
        if a.level == t:
            return a
        assert a.level > t
        return self.lincomb([(a, 1.0)], t)
