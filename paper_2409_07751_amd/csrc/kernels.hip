// HIP kernels of the RNS-CKKS ring layer for gfx950 (CDNA4, wave64).
//
// Words are 64-bit residues modulo primes below 2^61.  Three reductions are
// used, each where it is cheapest on the integer VALU:
//   * Shoup's precomputed-quotient product for multiplications by a constant
//     (NTT twiddles, basis-conversion scalars, q_l^-1, P^-1);
//   * Barrett with a per-prime shift for variable x variable products
//     (the ciphertext tensor, key generation);
//   * Montgomery REDC after 128-bit lazy accumulation for sums of products with
//     operands stored in Montgomery form (key-switch inner product, plaintext
//     linear combinations, basis conversion).
// All polynomials are limb-major: limb l of polynomial p of a set starts at
// base + l*lstride + p*pstride and holds N contiguous residues.
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

__device__ __forceinline__ int set_limb(int li, int skip_lo, int skip_hi)
{
    return li < skip_lo ? li : li + (skip_hi - skip_lo);
}

// ------------------------------------------------------------------------ NTT
// Negacyclic Cooley-Tukey NTT with the psi twist merged into the twiddles
// (bit-reversed psi powers): natural-order input, bit-reversed output; the
// inverse is Gentleman-Sande with N^-1 fused into its last store.
//
// N = R * C with C = 2^min(logN, 8).  Pass 1 runs the first log R stages on
// columns (elements c, c+C, c+2C, ...), a 2048-word tile of TC adjacent
// columns per workgroup; pass 2 runs the last log C stages on contiguous
// rows of C words, RB rows per workgroup.  Inside a pass each thread holds a
// radix-8 unit (three stages) in registers; units are exchanged through LDS
// between phases, so a pass costs two LDS round trips instead of one per
// stage.  The first phase reads global memory and the last writes it.
// Butterflies are Harvey's lazy ones: forward values stay in [0, 4q),
// inverse values in [0, 2q), and only the final store reduces to [0, q).

template <int LOGN>
struct NttGeo {
    static constexpr int LC = LOGN < 8 ? LOGN : 8;
    static constexpr int LR = LOGN - LC;
    static constexpr int LTC = (11 - LR) < LC ? (11 - LR) : LC;
    static constexpr int LRB = (11 - LC) < LR ? (11 - LC) : LR;
};

__device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 wp, u64 q) { return a * w - __umul64hi(a, wp) * q; }

// X, Y in [0, 4q) -> [0, 4q)
__device__ __forceinline__ void ct_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q2)
{
    u64 x = X >= q2 ? X - q2 : X;
    u64 t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + q2;
}

// X, Y in [0, 2q) -> [0, 2q)
__device__ __forceinline__ void gs_bfly(u64 &X, u64 &Y, u64 w, u64 wp, u64 q, u64 q2)
{
    u64 s = X + Y;
    s = s >= q2 ? s - q2 : s;
    u64 t = X - Y + q2;
    X = s;
    Y = shoup_lazy(t, w, wp, q);
}

enum { SRC_GLOBAL = 0, SRC_LDS = 1 };
enum { OUT_LDS = 0, OUT_LAZY = 1, OUT_REDUCE4 = 2, OUT_SCALE = 3 };

// One phase of R stages (min distance 2^LS positions) over a tile of
// 2^LP positions x 2^LL lines.  PASS 1: positions are rows, lines columns;
// PASS 2: positions are words of a row, lines rows.
template <int LOGN, int PASS, bool FWD, int R, int LS, int SRC, int OUT>
__device__ __forceinline__ void ntt_phase(u64 *sh, u64 *a, long blk, const u64 *w, const u64 *wp,
                                          const PrimeConst &pc)
{
    typedef NttGeo<LOGN> G;
    constexpr int LP = PASS == 1 ? G::LR : G::LC;
    constexpr int LL = PASS == 1 ? G::LTC : G::LRB;
    constexpr int LU = LP - R + LL;
    constexpr int LHI = LP - LS - R;
    constexpr int LG = PASS == 1 ? LS + G::LC : LS;  // log2 of the global stride of a unit
    const u64 q = pc.q, q2 = 2 * q;
    const long N = 1l << LOGN;
#pragma unroll
    for (int it = 0; it < ((1 << LU) + 255) / 256; it++) {
        const int u = it * 256 + (int)threadIdx.x;
        if ((1 << LU) % 256 != 0 && u >= (1 << LU)) break;
        int lo, hi, line;
        if (PASS == 1) {
            line = u & ((1 << LL) - 1);
            const int v = u >> LL;
            lo = v & ((1 << LS) - 1);
            hi = v >> LS;
        } else {
            lo = u & ((1 << LS) - 1);
            const int v = u >> LS;
            hi = v & ((1 << LHI) - 1);
            line = v >> LHI;
        }
        const int p0 = (hi << (LS + R)) | lo;
        // global index of position p on this line; LDS index
        auto gidx = [&](int p) -> long {
            return PASS == 1 ? ((long)p << G::LC) + (blk << G::LTC) + line
                             : (((blk << G::LRB) + line) << G::LC) + p;
        };
        auto lidx = [&](int p) -> int { return PASS == 1 ? (p << LL) + line : (line << LP) + p; };
        u64 x[1 << R];
#pragma unroll
        for (int k = 0; k < (1 << R); k++) {
            const int p = p0 + (k << LS);
            x[k] = SRC == SRC_GLOBAL ? a[gidx(p)] : sh[lidx(p)];
        }
        if (FWD) {
#pragma unroll
            for (int h = R - 1; h >= 0; h--) {
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = (N + gidx(p0 + (k << LS))) >> (LG + h + 1);
                    ct_bfly(x[k], x[k + (1 << h)], w[idx], wp[idx], q, q2);
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < R; h++) {
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = (N + gidx(p0 + (k << LS))) >> (LG + h + 1);
                    gs_bfly(x[k], x[k + (1 << h)], w[idx], wp[idx], q, q2);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < (1 << R); k++) {
            const int p = p0 + (k << LS);
            u64 v = x[k];
            if (OUT == OUT_LDS) {
                sh[lidx(p)] = v;
                continue;
            }
            if (OUT == OUT_REDUCE4) {
                v = v >= q2 ? v - q2 : v;
                v = v >= q ? v - q : v;
            } else if (OUT == OUT_SCALE) {
                v = shoup_lazy(v, pc.ninv, pc.ninvp, q);
                v = v >= q ? v - q : v;
            }
            a[gidx(p)] = v;
        }
    }
}

// phase plan: forward 3,3,..,rem; inverse rem,..,3,3
template <int LP, bool FWD, int PH>
struct PhasePlan {
    static constexpr int NPH = (LP + 2) / 3;
    static constexpr int REM = LP - 3 * (NPH - 1);
    static constexpr int R = FWD ? (PH < NPH - 1 ? 3 : REM) : (PH == 0 ? REM : 3);
    static constexpr int BEFORE = FWD ? 3 * PH : (PH == 0 ? 0 : REM + 3 * (PH - 1));
    static constexpr int LS = FWD ? LP - BEFORE - R : BEFORE;
};

template <int LOGN, int PASS, bool FWD, int PH, int LAST_OUT>
__device__ __forceinline__ void ntt_phases(u64 *sh, u64 *a, long blk, const u64 *w, const u64 *wp,
                                           const PrimeConst &pc)
{
    typedef NttGeo<LOGN> G;
    constexpr int LP = PASS == 1 ? G::LR : G::LC;
    typedef PhasePlan<LP, FWD, PH> P;
    constexpr bool first = PH == 0, last = PH == P::NPH - 1;
    constexpr int SRC = first ? SRC_GLOBAL : SRC_LDS;
    constexpr int OUT = last ? LAST_OUT : OUT_LDS;
    ntt_phase<LOGN, PASS, FWD, P::R, P::LS, SRC, OUT>(sh, a, blk, w, wp, pc);
    if constexpr (!last) {
        __syncthreads();
        ntt_phases<LOGN, PASS, FWD, PH + 1, LAST_OUT>(sh, a, blk, w, wp, pc);
    }
}

template <int LOGN, int PASS, bool FWD, int LAST_OUT>
__global__ void __launch_bounds__(256) k_ntt(NttTables T, PolySet ps, LimbMap lm, int skip_lo, int skip_hi)
{
    typedef NttGeo<LOGN> G;
    constexpr int LT = PASS == 1 ? G::LR + G::LTC : G::LC + G::LRB;
    __shared__ u64 sh[1 << LT];
    const int y = blockIdx.y;
    const int poly = y % ps.npoly;
    const int limb = set_limb(y / ps.npoly, skip_lo, skip_hi);
    const int pi = lm.prime(limb);
    const PrimeConst pc = T.pc[pi];
    u64 *a = ps.base + (long)limb * ps.lstride + (long)poly * ps.pstride;
    const u64 *w = (FWD ? T.fw : T.iw) + ((long)pi << LOGN);
    const u64 *wp = (FWD ? T.fwp : T.iwp) + ((long)pi << LOGN);
    ntt_phases<LOGN, PASS, FWD, 0, LAST_OUT>(sh, a, (long)blockIdx.x, w, wp, pc);
}

template <int LOGN>
static void ntt_launch_n(const NttTables &t, PolySet ps, LimbMap lm, int skip_lo, int skip_hi, bool inverse,
                         int nl, hipStream_t s, KernelTimer *tm)
{
    typedef NttGeo<LOGN> G;
    dim3 blk(256);
    dim3 g1(1 << (G::LC - G::LTC), nl * ps.npoly);
    dim3 g2(1 << (G::LR - G::LRB), nl * ps.npoly);
    // algorithmic work of one pass: every word read and written once, N/2
    // butterflies per stage
    const double polys = (double)nl * ps.npoly;
    const double bytes = 16.0 * (double)(1l << LOGN) * polys;
    const double b1 = polys * (double)(1l << (LOGN - 1)) * G::LR, b2 = polys * (double)(1l << (LOGN - 1)) * G::LC;
    auto timed = [&](int id, double ops, auto launch) {
        bool on = tm && tm->on(id);
        if (on) tm->before(s);
        launch();
        if (on) tm->after(s, bytes, ops);
    };
    if constexpr (G::LR > 0) {
        if (!inverse) {
            timed(KID_NTT_FWD1, b1, [&] {
                hipLaunchKernelGGL((k_ntt<LOGN, 1, true, OUT_LAZY>), g1, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
            });
            timed(KID_NTT_FWD2, b2, [&] {
                hipLaunchKernelGGL((k_ntt<LOGN, 2, true, OUT_REDUCE4>), g2, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
            });
        } else {
            timed(KID_NTT_INV2, b2, [&] {
                hipLaunchKernelGGL((k_ntt<LOGN, 2, false, OUT_LAZY>), g2, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
            });
            timed(KID_NTT_INV1, b1, [&] {
                hipLaunchKernelGGL((k_ntt<LOGN, 1, false, OUT_SCALE>), g1, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
            });
        }
    } else {
        (void)g1;
        if (!inverse)
            hipLaunchKernelGGL((k_ntt<LOGN, 2, true, OUT_REDUCE4>), g2, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
        else
            hipLaunchKernelGGL((k_ntt<LOGN, 2, false, OUT_SCALE>), g2, blk, 0, s, t, ps, lm, skip_lo, skip_hi);
    }
}

void launch_ntt(const NttTables &t, PolySet ps, LimbMap lm, int skip_lo, int skip_hi, bool inverse,
                hipStream_t s, KernelTimer *tm)
{
    int nl = ps.nl - (skip_hi - skip_lo);
    if (nl <= 0) return;
    switch (t.logN) {
    case 4: ntt_launch_n<4>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 5: ntt_launch_n<5>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 6: ntt_launch_n<6>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 7: ntt_launch_n<7>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 8: ntt_launch_n<8>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 9: ntt_launch_n<9>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 10: ntt_launch_n<10>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 11: ntt_launch_n<11>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 12: ntt_launch_n<12>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 13: ntt_launch_n<13>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 14: ntt_launch_n<14>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 15: ntt_launch_n<15>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    case 16: ntt_launch_n<16>(t, ps, lm, skip_lo, skip_hi, inverse, nl, s, tm); break;
    default: break;
    }
}

// ----------------------------------------------------------- elementwise ops
#define EW_INDEX                                                                   \
    int y = blockIdx.y;                                                            \
    int poly = y % a.npoly, limb = y / a.npoly;                                    \
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;                          \
    if (n >= N) return;

__global__ void k_addsub(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int op, int N)
{
    EW_INDEX
    u64 q = pc[lm.prime(limb)].q;
    u64 x = a.base[limb * a.lstride + poly * a.pstride + n];
    u64 z = b.base[limb * b.lstride + poly * b.pstride + n];
    out.base[limb * out.lstride + poly * out.pstride + n] = op == 0 ? addm(x, z, q) : subm(x, z, q);
}

void launch_addsub(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int op, int N,
                   hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_addsub, g, dim3(256), 0, s, pc, out, a, b, lm, op, N);
}

__global__ void k_mul_scalar(const PrimeConst *pc, PolySet out, PolySet a, const u64 *ks, const u64 *ksp,
                             LimbMap lm, int N)
{
    EW_INDEX
    u64 q = pc[lm.prime(limb)].q;
    u64 x = a.base[limb * a.lstride + poly * a.pstride + n];
    out.base[limb * out.lstride + poly * out.pstride + n] = shoup(x, ks[limb], ksp[limb], q);
}

void launch_mul_scalar(const PrimeConst *pc, PolySet out, PolySet a, const u64 *ks, const u64 *ksp,
                       LimbMap lm, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_mul_scalar, g, dim3(256), 0, s, pc, out, a, ks, ksp, lm, N);
}

__global__ void k_add_const(const PrimeConst *pc, PolySet a, const u64 *c, LimbMap lm, int N)
{
    EW_INDEX
    if (poly != 0) return;
    u64 q = pc[lm.prime(limb)].q;
    u64 *p = a.base + limb * a.lstride + n;
    *p = addm(*p, c[limb], q);
}

void launch_add_const(const PrimeConst *pc, PolySet a, const u64 *c, LimbMap lm, int N, hipStream_t s)
{
    PolySet a1 = a;
    a1.npoly = 1;
    dim3 g((N + 255) / 256, a.nl);
    hipLaunchKernelGGL(k_add_const, g, dim3(256), 0, s, pc, a1, c, lm, N);
}

// d: [limb][3][N] (pstride), a, b: two polynomials each
__global__ void k_tensor(const PrimeConst *pc, PolySet d, PolySet a, PolySet b, LimbMap lm, int N, int acc)
{
    int limb = blockIdx.y;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[lm.prime(limb)];
    const u64 *pa = a.base + limb * a.lstride + n, *pb = b.base + limb * b.lstride + n;
    u64 a0 = pa[0], a1 = pa[a.pstride], b0 = pb[0], b1 = pb[b.pstride];
    u64 d0 = barrett(a0, b0, c);
    u64 d1 = addm(barrett(a0, b1, c), barrett(a1, b0, c), c.q);
    u64 d2 = barrett(a1, b1, c);
    u64 *pd = d.base + limb * d.lstride + n;
    if (acc) {
        d0 = addm(d0, pd[0], c.q);
        d1 = addm(d1, pd[d.pstride], c.q);
        d2 = addm(d2, pd[2 * d.pstride], c.q);
    }
    pd[0] = d0;
    pd[d.pstride] = d1;
    pd[2 * d.pstride] = d2;
}

void launch_tensor(const PrimeConst *pc, PolySet d, PolySet a, PolySet b, LimbMap lm, int N, bool acc,
                   hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl);
    hipLaunchKernelGGL(k_tensor, g, dim3(256), 0, s, pc, d, a, b, lm, N, acc ? 1 : 0);
}

#define LC_MAX 16
struct LcArgs {
    const u64 *a[LC_MAX];
    const u64 *pt[LC_MAX];
    int is_const[LC_MAX];
};

__global__ void k_lincomb(const PrimeConst *pc, PolySet out, LcArgs args, long a_lstride, long a_pstride,
                          long pt_lstride, int nterms, LimbMap lm, int N)
{
    int y = blockIdx.y;
    int poly = y % out.npoly, limb = y / out.npoly;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[lm.prime(limb)];
    u64 lo = 0, hi = 0;
    for (int k = 0; k < nterms; k++) {
        u64 x = args.a[k][limb * a_lstride + poly * a_pstride + n];
        u64 p = args.is_const[k] ? args.pt[k][limb] : args.pt[k][limb * pt_lstride + n];
        mac(lo, hi, x, p);
    }
    out.base[limb * out.lstride + poly * out.pstride + n] = redc(lo, hi, c);
}

void launch_lincomb(const PrimeConst *pc, PolySet out, const u64 *const *a_bases, long a_lstride,
                    long a_pstride, const u64 *const *pt_bases, long pt_lstride, int nterms, LimbMap lm,
                    int N, hipStream_t s)
{
    LcArgs args;
    for (int k = 0; k < nterms; k++) {
        args.a[k] = a_bases[k];
        // a constant term is tagged by the low bit of its pointer
        uintptr_t v = (uintptr_t)pt_bases[k];
        args.is_const[k] = (int)(v & 1);
        args.pt[k] = (const u64 *)(v & ~(uintptr_t)1);
    }
    dim3 g((N + 255) / 256, out.nl * out.npoly);
    hipLaunchKernelGGL(k_lincomb, g, dim3(256), 0, s, pc, out, args, a_lstride, a_pstride, pt_lstride,
                       nterms, lm, N);
}

__global__ void k_automorph(PolySet out, PolySet a, u64 g, int logN)
{
    int y = blockIdx.y;
    int poly = y % a.npoly, limb = y / a.npoly;
    u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (1u << logN)) return;
    out.base[limb * out.lstride + poly * out.pstride + j] =
        a.base[limb * a.lstride + poly * a.pstride + auto_src(j, g, logN)];
}

void launch_automorph(PolySet out, PolySet a, u64 g, int logN, hipStream_t s)
{
    int N = 1 << logN;
    dim3 gr((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_automorph, gr, dim3(256), 0, s, out, a, g, logN);
}

__global__ void k_copy(PolySet out, PolySet a, int N)
{
    EW_INDEX
    out.base[limb * out.lstride + poly * out.pstride + n] = a.base[limb * a.lstride + poly * a.pstride + n];
}

void launch_copy(PolySet out, PolySet in, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, in.nl * in.npoly);
    hipLaunchKernelGGL(k_copy, g, dim3(256), 0, s, out, in, N);
}

__global__ void k_pmul(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int N)
{
    EW_INDEX
    const PrimeConst &c = pc[lm.prime(limb)];
    u64 x = a.base[limb * a.lstride + poly * a.pstride + n];
    u64 z = b.base[limb * b.lstride + poly * b.pstride + n];
    out.base[limb * out.lstride + poly * out.pstride + n] = barrett(x, z, c);
}

void launch_pmul(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_pmul, g, dim3(256), 0, s, pc, out, a, b, lm, N);
}

// ------------------------------------------------------------------ rescale
// last: limb l of each polynomial in coefficient form (npoly polys, 1 limb);
// tmp[i][p] = ([last + h]_{q_l} - h) mod q_i for i < l, h = floor(q_l / 2)
__global__ void k_rescale_prep(const PrimeConst *pc, PolySet tmp, PolySet last, int l, int N)
{
    int y = blockIdx.y;
    int poly = y % tmp.npoly, i = y / tmp.npoly;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    u64 ql = pc[l].q, h = ql >> 1;
    const PrimeConst &c = pc[i];
    u64 r = addm(last.base[poly * last.pstride + n], h, ql);
    u64 hi = reduce64(h, c);
    tmp.base[i * tmp.lstride + poly * tmp.pstride + n] = subm(reduce64(r, c), hi, c.q);
}

void launch_rescale_prep(const PrimeConst *pc, PolySet tmp_out, PolySet last_coeff, int l, int N,
                         hipStream_t s)
{
    dim3 g((N + 255) / 256, l * tmp_out.npoly);
    hipLaunchKernelGGL(k_rescale_prep, g, dim3(256), 0, s, pc, tmp_out, last_coeff, l, N);
}

__global__ void k_rescale_fin(const PrimeConst *pc, PolySet out, PolySet in, PolySet t, const u64 *inv,
                              const u64 *invp, int N)
{
    int y = blockIdx.y;
    int poly = y % out.npoly, i = y / out.npoly;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    u64 q = pc[i].q;
    u64 x = in.base[i * in.lstride + poly * in.pstride + n];
    u64 z = t.base[i * t.lstride + poly * t.pstride + n];
    out.base[i * out.lstride + poly * out.pstride + n] = shoup(subm(x, z, q), inv[i], invp[i], q);
}

void launch_rescale_fin(const PrimeConst *pc, PolySet out, PolySet in, PolySet t, const u64 *inv,
                        const u64 *invp, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, out.nl * out.npoly);
    hipLaunchKernelGGL(k_rescale_fin, g, dim3(256), 0, s, pc, out, in, t, inv, invp, N);
}

// ------------------------------------------------------- basis conversion
// out_t = REDC( sum_j [x_j * invhat_j]_{q_j} * hatm_{j,t} ),  hatm in Montgomery form
// Every thread converts one coefficient for a chunk of BC_TCH target limbs.
#define BC_TCH 4
__global__ void k_bconv(const PrimeConst *pc, BconvPlan plan, const u64 *src, long src_ls, u64 *dst,
                        long dst_ls, int N)
{
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    u64 y[8];
    for (int j = 0; j < plan.ns; j++) {
        const PrimeConst &c = pc[plan.src_prime[j]];
        y[j] = shoup(src[j * src_ls + n], plan.invhat[j], plan.invhatp[j], c.q);
    }
    int t0 = blockIdx.y * BC_TCH;
    int t1 = t0 + BC_TCH < plan.nd ? t0 + BC_TCH : plan.nd;
    for (int t = t0; t < t1; t++) {
        const PrimeConst &c = pc[plan.dst_prime[t]];
        u64 lo = 0, hi = 0;
        for (int j = 0; j < plan.ns; j++) mac(lo, hi, y[j], plan.hatm[j * plan.nd + t]);
        dst[plan.dst_limb[t] * dst_ls + n] = redc(lo, hi, c);
    }
}

void launch_bconv(const PrimeConst *pc, const BconvPlan &plan, const u64 *src, long src_lstride, u64 *dst,
                  long dst_lstride, int N, hipStream_t s, KernelTimer *tm)
{
    dim3 g((N + 255) / 256, (plan.nd + BC_TCH - 1) / BC_TCH);
    bool on = tm && tm->on(KID_BCONV);
    if (on) tm->before(s);
    hipLaunchKernelGGL(k_bconv, g, dim3(256), 0, s, pc, plan, src, src_lstride, dst, dst_lstride, N);
    if (on) tm->after(s, 8.0 * N * (plan.ns + plan.nd), (double)N * plan.ns * plan.nd);
}

// ---------------------------------------------------- key-switch inner product
__global__ void k_keyip(const PrimeConst *pc, u64 *acc, long acc_pstride, const u64 *ext, long ext_dstride,
                        const u64 *key, long key_dstride, long key_cstride, int ndig, LimbMap lm,
                        int key_nq_off, u64 galois, int logN)
{
    int t = blockIdx.y;
    u32 n = blockIdx.x * blockDim.x + threadIdx.x;
    int N = 1 << logN;
    if (n >= (u32)N) return;
    const PrimeConst &c = pc[lm.prime(t)];
    int kt = t < lm.nq ? t : key_nq_off + (t - lm.nq);
    u32 src = galois > 1 ? auto_src(n, galois, logN) : n;
    u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
    for (int j = 0; j < ndig; j++) {
        u64 e = ext[j * ext_dstride + (long)t * N + src];
        const u64 *kp = key + j * key_dstride + (long)kt * N + n;
        mac(lo0, hi0, e, kp[0]);
        mac(lo1, hi1, e, kp[key_cstride]);
    }
    acc[(long)t * N + n] = redc(lo0, hi0, c);
    acc[acc_pstride + (long)t * N + n] = redc(lo1, hi1, c);
}

void launch_keyip(const PrimeConst *pc, u64 *acc, long acc_pstride, const u64 *ext, long ext_dstride,
                  const u64 *key, long key_dstride, long key_cstride, int ndig, int nl, LimbMap lm,
                  int key_nq_off, u64 galois, int logN, hipStream_t s, KernelTimer *tm)
{
    int N = 1 << logN;
    dim3 g((N + 255) / 256, nl);
    bool on = tm && tm->on(KID_KEYIP);
    if (on) tm->before(s);
    hipLaunchKernelGGL(k_keyip, g, dim3(256), 0, s, pc, acc, acc_pstride, ext, ext_dstride, key, key_dstride,
                       key_cstride, ndig, lm, key_nq_off, galois, logN);
    // reads ndig extended digits and 2 ndig key polynomials, writes 2 outputs
    if (on) tm->after(s, 8.0 * N * nl * (3.0 * ndig + 2.0), 2.0 * N * nl * ndig);
}

// ModDown tail on Q limbs: out_c = base_c + (acc_c - conv_c) * P^-1
__global__ void k_moddown_fin(const PrimeConst *pc, PolySet out, PolySet base, int has_base0, int has_base1,
                              u64 g0, const u64 *acc, long acc_ls, long acc_ps, const u64 *conv, long conv_ls,
                              long conv_ps, const u64 *pinv, const u64 *pinvp, int logN)
{
    int y = blockIdx.y;
    int poly = y & 1, i = y >> 1;
    u32 n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (1u << logN)) return;
    u64 q = pc[i].q;
    u64 v = subm(acc[i * acc_ls + poly * acc_ps + n], conv[i * conv_ls + poly * conv_ps + n], q);
    v = shoup(v, pinv[i], pinvp[i], q);
    int has = poly == 0 ? has_base0 : has_base1;
    if (has) {
        u32 src = (poly == 0 && g0 > 1) ? auto_src(n, g0, logN) : n;
        v = addm(v, base.base[i * base.lstride + poly * base.pstride + src], q);
    }
    out.base[i * out.lstride + poly * out.pstride + n] = v;
}

void launch_moddown_fin(const PrimeConst *pc, PolySet out, PolySet base, int base_mask, u64 galois,
                        const u64 *acc, long acc_lstride, long acc_pstride, const u64 *conv,
                        long conv_lstride, long conv_pstride, const u64 *pinv, const u64 *pinvp, int logN,
                        hipStream_t s)
{
    int N = 1 << logN;
    dim3 g((N + 255) / 256, out.nl * 2);
    hipLaunchKernelGGL(k_moddown_fin, g, dim3(256), 0, s, pc, out, base, base_mask & 1, (base_mask >> 1) & 1,
                       galois, acc, acc_lstride, acc_pstride, conv, conv_lstride,
                       conv_pstride, pinv, pinvp, logN);
}

// -------------------------------------------------------- keys and client ops
// b = e - a s + pfac * s' (NTT domain, standard form), then both b and a are
// converted to Montgomery form for the inner product
__global__ void k_keygen_b(const PrimeConst *pc, u64 *b, u64 *a, const u64 *s, const u64 *e, const u64 *sp,
                           const u64 *pfac, int N)
{
    int t = blockIdx.y;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[t];
    long o = (long)t * N + n;
    u64 as = barrett(a[o], s[o], c);
    u64 v = subm(e[o], as, c.q);
    if (pfac[t]) v = addm(v, barrett(pfac[t], sp[o], c), c.q);
    b[o] = shoup(v, c.r1, c.r1p, c.q);
    a[o] = shoup(a[o], c.r1, c.r1p, c.q);
}

void launch_keygen_b(const PrimeConst *pc, u64 *b, const u64 *a, const u64 *s, const u64 *e, const u64 *sp,
                     const u64 *pfac, int ntot, int N, hipStream_t st)
{
    dim3 g((N + 255) / 256, ntot);
    hipLaunchKernelGGL(k_keygen_b, g, dim3(256), 0, st, pc, b, (u64 *)a, s, e, sp, pfac, N);
}

__global__ void k_to_mont(const PrimeConst *pc, u64 *x, long ls, long ps_, int npoly, LimbMap lm, int N)
{
    int y = blockIdx.y;
    int poly = y % npoly, limb = y / npoly;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[lm.prime(limb)];
    u64 *p = x + limb * ls + poly * ps_ + n;
    *p = shoup(*p, c.r1, c.r1p, c.q);
}

void launch_to_montgomery(const PrimeConst *pc, u64 *x, long lstride, int nl, LimbMap lm, int N, int npoly,
                          long pstride, hipStream_t s)
{
    dim3 g((N + 255) / 256, nl * npoly);
    hipLaunchKernelGGL(k_to_mont, g, dim3(256), 0, s, pc, x, lstride, pstride, npoly, lm, N);
}

__global__ void k_decrypt0(const PrimeConst *pc, u64 *m, const u64 *c0, const u64 *c1, const u64 *s, int N)
{
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[0];
    m[n] = addm(c0[n], barrett(c1[n], s[n], c), c.q);
}

void launch_decrypt0(const PrimeConst *pc, u64 *m, const u64 *c0, const u64 *c1, const u64 *s, int N,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_decrypt0, dim3((N + 255) / 256), dim3(256), 0, st, pc, m, c0, c1, s, N);
}

// c0 = em - a s  (em = e + m, NTT domain); c0 and a are the two polynomials
// of limb l of the ciphertext (lstride c_lstride), s is [l][N]
__global__ void k_encrypt(const PrimeConst *pc, u64 *c0, const u64 *a, const u64 *s, const u64 *em,
                          long c_ls, int N)
{
    int l = blockIdx.y;
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[l];
    u64 as = barrett(a[l * c_ls + n], s[(long)l * N + n], c);
    c0[l * c_ls + n] = subm(em[(long)l * N + n], as, c.q);
}

void launch_encrypt(const PrimeConst *pc, u64 *c0, const u64 *a, const u64 *s, const u64 *em, long c_lstride,
                    int nl, int N, hipStream_t st)
{
    dim3 g((N + 255) / 256, nl);
    hipLaunchKernelGGL(k_encrypt, g, dim3(256), 0, st, pc, c0, a, s, em, c_lstride, N);
}

}  // namespace hk
