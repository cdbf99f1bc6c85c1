// Device-side modular arithmetic on 64-bit words (primes below 2^61).
#pragma once
#include "dev.hpp"

namespace hk {

// ------------------------------------------------------------ modular helpers
__device__ __forceinline__ u64 addm(u64 a, u64 b, u64 q)
{
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// a * w mod q with wp = floor(w 2^64 / q); valid for any 64-bit a, w < q < 2^63
__device__ __forceinline__ u64 shoup(u64 a, u64 w, u64 wp, u64 q)
{
    u64 h = __umul64hi(a, wp);
    u64 r = a * w - h * q;
    return r >= q ? r - q : r;
}

// a * b mod q for a*b < 2^(2b), b = bit length of q (HAC 14.42 with base 2)
__device__ __forceinline__ u64 barrett(u64 a, u64 b, const PrimeConst &c)
{
    u64 lo = a * b, hi = __umul64hi(a, b);
    int nb = c.bits;
    u64 z1 = (lo >> (nb - 1)) | (hi << (65 - nb));
    u64 plo = z1 * c.mu, phi = __umul64hi(z1, c.mu);
    u64 qh = (plo >> (nb + 1)) | (phi << (63 - nb));
    u64 r = lo - qh * c.q;
    if (r >= c.q) r -= c.q;
    if (r >= c.q) r -= c.q;
    return r;
}

// reduce a 64-bit value below 2^(2b)
__device__ __forceinline__ u64 reduce64(u64 a, const PrimeConst &c) { return barrett(a, 1, c); }

__device__ __forceinline__ void mac(u64 &lo, u64 &hi, u64 a, u64 b)
{
    u64 pl = a * b, ph = __umul64hi(a, b);
    lo += pl;
    hi += ph + (lo < pl ? 1ull : 0ull);
}

// (hi:lo) * 2^-64 mod q for (hi:lo) < q 2^64
__device__ __forceinline__ u64 redc(u64 lo, u64 hi, const PrimeConst &c)
{
    u64 m = lo * c.qinv_neg;
    u64 t = hi + __umul64hi(m, c.q) + (lo != 0 ? 1ull : 0ull);
    return t >= c.q ? t - c.q : t;
}

__device__ __forceinline__ u32 brv(u32 x, int bits) { return __brev(x) >> (32 - bits); }

// index of the NTT slot that sigma_g moves to slot j: slot j holds the
// evaluation at psi^(2 brv(j) + 1)
__device__ __forceinline__ u32 auto_src(u32 j, u64 g, int logN)
{
    u64 twoN = 2ull << logN;
    u64 e = (2ull * brv(j, logN) + 1ull) * g & (twoN - 1);
    return brv((u32)((e - 1) >> 1), logN);
}

__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wp, u64 q) { return a * w - __umul64hi(a, wp) * q; }

// ------------------------------------------------- exact FP64 residue arithmetic
// For q < 2^46 a residue, and every intermediate below, is an integer held
// exactly in a double; FP64 FMA runs at the full vector rate while 64-bit
// integer multiplies take several instructions.  Values are kept in a signed
// ("balanced") range and reduced only when they leave the transform.
// These helpers are host-callable as well (compiler builtins only, the same
// IEEE operations on both sides), so the bounds below can be checked on the
// CPU against exact integer arithmetic.

// u64 below 2^52 -> the same integer as a double
__host__ __device__ __forceinline__ double u2d(u64 v)
{
    return __builtin_bit_cast(double, v | 0x4330000000000000ull) - 4503599627370496.0;
}

// the bits of a double holding an integer in [0, 2^52) -> that integer
__device__ __forceinline__ u64 d2u_exact(u64 bits)
{
    return (u64)__double_as_longlong(__longlong_as_double((long long)bits) + 4503599627370496.0) & 0xFFFFFFFFFFFFFull;
}

// integer-valued double with |v| < 2^52 -> v mod q in [0, q)
__host__ __device__ __forceinline__ u64 d2u_mod(double v, double q, double qi)
{
    double r = __builtin_fma(-__builtin_rint(v * qi), q, v);  // exact, |r| <= q/2 + 1
    r = r < 0.0 ? r + q : r;
    return __builtin_bit_cast(u64, r + 4503599627370496.0) & 0xFFFFFFFFFFFFFull;
}

// y w mod q up to sign, |result| <= 3q/4, for |y| <= 2^50, |w| < q < 2^46,
// c = w / q rounded (fl(w / q), or fl(w fl(1 / q)) for a twiddle formed on
// the fly): the quotient estimate t = rint(y c) is within 3/4 of y w / q,
// p + e = y w exactly (e = the rounding error of p, exact by FMA), and
// p - t q is an integer below 2^47 in magnitude, so the FMA is exact too
__host__ __device__ __forceinline__ double mulm_fp(double y, double w, double c, double q)
{
    const double t = __builtin_rint(y * c);
    const double p = y * w;
    const double e = __builtin_fma(y, w, -p);
    return __builtin_fma(-t, q, p) + e;
}

}  // namespace hk
