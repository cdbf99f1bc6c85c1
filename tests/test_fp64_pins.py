"""CPU pins of the product's exact FP64 residue arithmetic (primes below 2^46).

The GPU transforms, basis conversions and rescale tails of the scale primes
compute residues in FP64: mulm_fp(y, w, c, q) forms y w mod q up to sign as
rint(y c), y w and its FMA rounding error, d2u_mod reduces an integer-valued
double into [0, q), and a forward transform adds each butterfly's product
without reduction.  Bit-exact parity with the integer oracle rests on three
claims: mulm_fp is exact mod q with |result| <= 3q/4 for |y| <= 2^50 and
|w| < q (c = fl(w/q), or W fl(1/q) for a twiddle formed on the fly with
|W| <= 3q/4); d2u_mod is exact for |v| < 2^52; and a forward transform whose
inputs are below 4q in magnitude stays within 16q <= 2^50.  These tests call
the product's own helpers, compiled for the host from the same header the
kernels use (tests/fp64/fp64_pin.hip), and check them against Python integer
arithmetic for primes of 40, 45 and 46 bits at random and worst-case
magnitudes, plus one whole N = 2^16 forward transform with the GPU's
butterfly and twiddle arithmetic against an exact integer transform."""
import ctypes
import os
import random
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fp64", "fp64_pin.hip")
HDR = os.path.join(HERE, "..", "paper_2409_07751_amd", "csrc", "modarith.hpp")
BUILD = os.path.join(HERE, "fp64", "_build")
LIB = os.path.join(BUILD, "libfp64pin.so")
LOGN = 16
N = 1 << LOGN

_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):  # deterministic below 3.3e24
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def prime_below(bits, m=2 * N):
    """The largest prime q = 1 mod m below 2^bits."""
    q = ((1 << bits) - 1) // m * m + 1
    while not _is_prime(q):
        q -= m
    return q


PRIMES = [prime_below(40), prime_below(45), prime_below(46)]


@pytest.fixture(scope="module")
def lib():
    os.makedirs(BUILD, exist_ok=True)
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(HDR)):
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run([hipcc, "-x", "hip", "-std=c++17", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                        "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        SRC, "-o", tmp], check=True, capture_output=True)
        os.replace(tmp, LIB)
    L = ctypes.CDLL(LIB)
    L.fp_mulm.argtypes = [_dp, _dp, _dp, ctypes.c_double, _dp, ctypes.c_size_t]
    L.fp_d2u_mod.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _u64p, ctypes.c_size_t]
    L.fp_u2d.argtypes = [_u64p, _dp, ctypes.c_size_t]
    L.fp_forward_ntt.argtypes = [_dp, ctypes.c_int, ctypes.c_double, _u64p, _u64p, _u64p, _u64p, _dp]
    for f in (L.fp_mulm, L.fp_d2u_mod, L.fp_u2d, L.fp_forward_ntt):
        f.restype = None
    return L


def _d(a):
    return np.ascontiguousarray(a, np.float64)


def mulm(lib, y, w, c, q):
    y, w, c = _d(y), _d(w), _d(c)
    out = np.zeros(len(y))
    lib.fp_mulm(y.ctypes.data_as(_dp), w.ctypes.data_as(_dp), c.ctypes.data_as(_dp), float(q),
                out.ctypes.data_as(_dp), len(y))
    return out


def check_mulm(y, w, r, q):
    """r is an integer congruent to y w mod q with |r| <= 3q/4 (exact integers)."""
    for yi, wi, ri in zip(y, w, r):
        assert ri == int(ri), (yi, wi, ri)
        assert (int(ri) - int(yi) * int(wi)) % q == 0, (yi, wi, ri)
        assert 4 * abs(int(ri)) <= 3 * q, (yi, wi, ri)


@pytest.mark.parametrize("q", PRIMES)
def test_mulm_fp_exact_and_bounded(lib, q):
    rnd = random.Random(q)
    lim = 1 << 50
    # worst-case magnitudes: |y| = 2^50, w = q - 1, 0, 1, and values near q/2
    ys = [lim, -lim, lim - 1, -(lim - 1), 16 * q, -16 * q, q - 1, -(q - 1), 0, 1, -1]
    ws = [q - 1, 1, 0, q // 2, q // 2 + 1, q - 2]
    y = [a for a in ys for _ in ws] + [rnd.randint(-lim, lim) for _ in range(20000)]
    w = [b for _ in ys for b in ws] + [rnd.randrange(q) for _ in range(20000)]
    c = [float(b) / float(q) for b in w]  # fl(w / q), as the host tables hold it
    check_mulm(y, w, mulm(lib, y, w, c, q), q)


@pytest.mark.parametrize("q", PRIMES)
def test_mulm_fp_signed_twiddle(lib, q):
    """A twiddle formed on the fly is W = mulm_fp(A, B) (|W| <= 3q/4, either
    sign) with quotient constant W fl(1/q); products by it are exact too."""
    rnd = random.Random(q + 1)
    lim = 1 << 50
    A = [rnd.randrange(q) for _ in range(4000)] + [q - 1, 1, q // 2]
    B = [rnd.randrange(q) for _ in range(4000)] + [q - 1, q - 1, q - 1]
    W = mulm(lib, A, B, [float(b) / float(q) for b in B], q)
    check_mulm(A, B, W, q)
    qi = 1.0 / float(q)
    y = [rnd.randint(-lim, lim) for _ in W[:-3]] + [lim, -lim, lim]
    check_mulm(y, W, mulm(lib, y, W, [float(v) * qi for v in W], q), q)


@pytest.mark.parametrize("q", PRIMES)
def test_d2u_mod_and_u2d_exact(lib, q):
    rnd = random.Random(q + 2)
    lim = (1 << 52) - 1
    v = [lim, -lim, 0, 1, -1, q, -q, q - 1, -(q - 1), q // 2, -(q // 2), q // 2 + 1, 7 * q, -7 * q] + \
        [rnd.randint(-lim, lim) for _ in range(20000)]
    vd = _d(v)
    assert all(float(a) == a for a in v)
    out = np.zeros(len(v), np.uint64)
    lib.fp_d2u_mod(vd.ctypes.data_as(_dp), float(q), 1.0 / float(q), out.ctypes.data_as(_u64p), len(v))
    assert [int(o) for o in out] == [a % q for a in v]
    u = np.array([0, 1, lim, q - 1] + [rnd.randrange(1 << 52) for _ in range(1000)], np.uint64)
    d = np.zeros(len(u))
    lib.fp_u2d(u.ctypes.data_as(_u64p), d.ctypes.data_as(_dp), len(u))
    assert all(int(a) == int(b) for a, b in zip(u, d))


def _brv(k, bits):
    return int(format(k, "0%db" % bits)[::-1], 2)


def _psi(q):
    """A primitive 2N-th root of unity mod q."""
    for g in range(2, 1000):
        psi = pow(g, (q - 1) // (2 * N), q)
        if pow(psi, N, q) == q - 1:
            return psi
    raise AssertionError("no root")


def _tables(q):
    psi = _psi(q)
    fw = [pow(psi, _brv(k, LOGN), q) for k in range(N)]
    LR = LOGN - 8
    A = [0] * ((1 << LR) * 8)
    B = [0] * 256
    for sp in range(8):
        base = 1 << (LR + sp)
        for r in range(1 << LR):
            A[r * 8 + sp] = fw[base + (r << sp)]
        inv0 = pow(fw[base], q - 2, q)
        for u in range(1 << sp):
            B[(1 << sp) - 1 + u] = fw[base + u] * inv0 % q
    return psi, fw, A, B


def exact_ntt(x, fw, q):
    """The same decimation-in-time transform in exact integer arithmetic."""
    x = np.array([int(v) % q for v in x], dtype=object)
    for s in range(LOGN):
        m, half = 1 << s, N >> (s + 1)
        x = x.reshape(m, 2, half)
        w = np.array(fw[m:2 * m], dtype=object).reshape(m, 1)
        r = x[:, 1, :] * w % q
        a = x[:, 0, :].copy()
        x[:, 0, :] = (a + r) % q
        x[:, 1, :] = (a - r) % q
        x = x.reshape(N)
    return x


def test_exact_ntt_is_evaluation_at_odd_powers():
    """The integer reference transform: slot k holds the evaluation at
    psi^(2 brv(k) + 1) (checked on sampled slots of an N = 2^16 transform)."""
    q = PRIMES[0]
    psi, fw, _, _ = _tables(q)
    rnd = random.Random(5)
    x = [rnd.randrange(q) for _ in range(N)]
    y = exact_ntt(x, fw, q)
    for k in (0, 1, 2, 12345, N - 1):
        z = pow(psi, 2 * _brv(k, LOGN) + 1, q)
        acc, p = 0, 1
        for v in x:
            acc = (acc + v * p) % q
            p = p * z % q
        assert y[k] == acc


@pytest.mark.parametrize("q", PRIMES)
@pytest.mark.parametrize("pattern", ["random", "max", "balanced", "4q"])
def test_fp64_forward_transform_exact_within_16q(lib, q, pattern):
    psi, fw, A, B = _tables(q)
    rnd = random.Random(q + len(pattern))
    if pattern == "random":
        x = [rnd.randrange(q) for _ in range(N)]
    elif pattern == "max":
        x = [q - 1] * N
    elif pattern == "balanced":  # the conversion passes hand over |x| <= q/2 + 1
        x = [rnd.choice((-1, 1)) * (q // 2 + 1) for _ in range(N)]
    else:  # the largest start the growth bound allows
        x = [4 * q - 1 if i % 3 else -(4 * q - 1) for i in range(N)]
    xd = _d(x)
    out = np.zeros(N, np.uint64)
    peak = ctypes.c_double()
    u = lambda a: np.ascontiguousarray(a, np.uint64)
    fwa, Aa, Ba = u(fw), u(A), u(B)
    lib.fp_forward_ntt(xd.ctypes.data_as(_dp), LOGN, float(q), fwa.ctypes.data_as(_u64p), Aa.ctypes.data_as(_u64p),
                       Ba.ctypes.data_as(_u64p), out.ctypes.data_as(_u64p), ctypes.byref(peak))
    want = exact_ntt(x, fw, q)
    assert [int(v) for v in out] == [int(v) for v in want]
    assert peak.value <= 16 * q <= 1 << 50
