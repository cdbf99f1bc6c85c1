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
#include "modarith.hpp"

namespace hk {


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

__global__ void k_add_c0(const PrimeConst *pc, PolySet out, PolySet a, const u64 *kf, const u64 *kfp, const u64 *c,
                         const u64 *p, LimbMap lm, int N)
{
    EW_INDEX
    const u64 q = pc[lm.prime(limb)].q;
    u64 x = a.base[limb * a.lstride + poly * a.pstride + n];
    if (kf) x = shoup(x, kf[limb], kfp[limb], q);
    if ((poly & 1) == 0 && (c || p)) x = addm(x, c ? c[limb] : p[(long)limb * N + n], q);
    out.base[limb * out.lstride + poly * out.pstride + n] = x;
}

void launch_add_c0(const PrimeConst *pc, PolySet out, PolySet a, const u64 *kf, const u64 *kfp, const u64 *c,
                   const u64 *p, LimbMap lm, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_add_c0, g, dim3(256), 0, s, pc, out, a, kf, kfp, c, p, lm, N);
}

// batch element e of d holds (d0, d1, d2) at +0, +N, +2N; of a and b (c0, c1)
// at +0, +N; pstride is the element stride
__global__ void k_tensor(const PrimeConst *pc, PolySet d, PolySet a, PolySet b, LimbMap lm, int N, int acc)
{
    const int y = blockIdx.y;
    const int e = y % a.npoly, limb = y / a.npoly;
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[lm.prime(limb)];
    const u64 *pa = a.base + limb * a.lstride + e * a.pstride + n, *pb = b.base + limb * b.lstride + e * b.pstride + n;
    u64 a0 = pa[0], a1 = pa[N], b0 = pb[0], b1 = pb[N];
    u64 d0 = barrett(a0, b0, c);
    u64 d1 = addm(barrett(a0, b1, c), barrett(a1, b0, c), c.q);
    u64 d2 = barrett(a1, b1, c);
    u64 *pd = d.base + limb * d.lstride + e * d.pstride + n;
    if (acc) {
        d0 = addm(d0, pd[0], c.q);
        d1 = addm(d1, pd[N], c.q);
        d2 = addm(d2, pd[2 * N], c.q);
    }
    pd[0] = d0;
    pd[N] = d1;
    pd[2 * N] = d2;
}

void launch_tensor(const PrimeConst *pc, PolySet d, PolySet a, PolySet b, LimbMap lm, int N, bool acc,
                   hipStream_t s)
{
    dim3 g((N + 255) / 256, a.nl * a.npoly);
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

// One rotation's share of a sum of rotations with a single ModDown: out
// (the running sum of accumulators, polynomial 2 e + c over Q_l u P) [+]=
// sigma_g(a) limb by limb (NTT form: a permutation of the slots), and on
// component 0's Q limbs (limb < nq) also [P]_{q_limb} sigma_g(c0_e), which the
// division by P in ModDown turns into sigma_g(c0_e) exactly; a, c0 and out
// do not overlap
__global__ void k_automorph_acc(const PrimeConst *pc, PolySet out, PolySet a, PolySet c0, const u64 *pm,
                                const u64 *pmp, u64 g, int logN, LimbMap lm, int nq, int accumulate)
{
    const int y = blockIdx.y;
    const int poly = y % a.npoly, limb = y / a.npoly;
    const u32 j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (1u << logN)) return;
    const u32 src = auto_src(j, g, logN);
    const int pr = lm.prime(limb);
    const u64 q = pc[pr].q;
    u64 v = a.base[limb * a.lstride + poly * a.pstride + src];
    if ((poly & 1) == 0 && limb < nq)
        v = addm(v, shoup(c0.base[limb * c0.lstride + (poly >> 1) * c0.pstride + src], pm[pr], pmp[pr], q), q);
    u64 *o = out.base + limb * out.lstride + poly * out.pstride + j;
    *o = accumulate ? addm(*o, v, q) : v;
}

void launch_automorph_acc(const PrimeConst *pc, PolySet out, PolySet a, PolySet c0, const u64 *pm, const u64 *pmp,
                          u64 g, int logN, LimbMap lm, int nq, bool accumulate, hipStream_t s)
{
    const int N = 1 << logN;
    dim3 gr((N + 255) / 256, a.nl * a.npoly);
    hipLaunchKernelGGL(k_automorph_acc, gr, dim3(256), 0, s, pc, out, a, c0, pm, pmp, g, logN, lm, nq,
                       accumulate ? 1 : 0);
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

// ---------------------------------------------------- key-switch inner product
// One thread per (coefficient, limb): the 2 ndig key words of that coefficient
// are loaded once into registers and reused for every batch element, so the
// key is read from HBM once per launch whatever the batch size.  MAXD bounds
// ndig; with ndig <= 16 and q < 2^60 the 128-bit sums stay below q 2^64, as
// Montgomery reduction requires.
template <int MAXD>
__global__ void __launch_bounds__(256) k_keyip(const PrimeConst *pc, u64 *__restrict__ acc, long acc_pstride,
                                               long acc_bstride, const u64 *__restrict__ ext, long ext_dstride,
                                               long ext_bstride, const u64 *__restrict__ d, long d_ls,
                                               long d_bstride, const u64 *__restrict__ key, long key_dstride,
                                               long key_cstride, int ndig, int skip_lo, int skip_hi, int nq, int w,
                                               int nb, LimbMap lm, int key_nq_off, int logN)
{
    const int t = (int)blockIdx.y < skip_lo ? (int)blockIdx.y : (int)blockIdx.y + (skip_hi - skip_lo);
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long N = 1l << logN;
    if (n >= N) return;
    const PrimeConst &c = pc[lm.prime(t)];
    const int kt = t < lm.nq ? t : key_nq_off + (t - lm.nq);
    u64 k0[MAXD], k1[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; j++) {
        if (j < ndig) {
            const u64 *kp = key + j * key_dstride + kt * N + n;
            k0[j] = kp[0];
            k1[j] = kp[key_cstride];
        }
    }
    // the digit whose own limbs include t reads the input polynomial itself
    const int jown = t < nq ? t / w : -1;
#pragma unroll 2
    for (int b = 0; b < nb; b++) {
        const u64 *eb = ext + b * ext_bstride + t * N + n;
        u64 lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
#pragma unroll
        for (int j = 0; j < MAXD; j++) {
            if (j < ndig) {
                const u64 e = j == jown ? d[b * d_bstride + t * d_ls + n] : eb[j * ext_dstride];
                mac(lo0, hi0, e, k0[j]);
                mac(lo1, hi1, e, k1[j]);
            }
        }
        u64 *ab = acc + b * acc_bstride + t * N + n;
        ab[0] = redc(lo0, hi0, c);
        ab[acc_pstride] = redc(lo1, hi1, c);
    }
}

int launch_keyip(const PrimeConst *pc, u64 *acc, long acc_pstride, long acc_bstride, const u64 *ext,
                 long ext_dstride, long ext_bstride, const u64 *d, long d_ls, long d_bstride, const u64 *key,
                 long key_dstride, long key_cstride, int ndig, int nl, int skip_lo, int skip_hi, int nq, int w,
                 int nb, LimbMap lm, int key_nq_off, int logN, hipStream_t s, KernelTimer *tm)
{
    if (ndig < 1 || ndig > 16) return -1;
    const int N = 1 << logN;
    dim3 g((N + 255) / 256, nl);
    bool on = tm && tm->on(KID_KEYIP);
    if (on) tm->before(s);
#define KEYIP_ARGS                                                                                              \
    pc, acc, acc_pstride, acc_bstride, ext, ext_dstride, ext_bstride, d, d_ls, d_bstride, key, key_dstride,     \
        key_cstride, ndig, skip_lo, skip_hi, nq, w, nb, lm, key_nq_off, logN
    if (ndig <= 4) hipLaunchKernelGGL(k_keyip<4>, g, dim3(256), 0, s, KEYIP_ARGS);
    else if (ndig <= 8) hipLaunchKernelGGL(k_keyip<8>, g, dim3(256), 0, s, KEYIP_ARGS);
    else hipLaunchKernelGGL(k_keyip<16>, g, dim3(256), 0, s, KEYIP_ARGS);
#undef KEYIP_ARGS
    // reads nb ndig extended digits and 2 ndig key polynomials, writes 2 nb outputs
    if (on) tm->after(s, 8.0 * N * nl * (nb * ndig + 2.0 * ndig + 2.0 * nb), 2.0 * N * nl * ndig * nb);
    return 0;
}

__global__ void k_key_fp(const PrimeConst *pc, const u64 *kmont, u64 *kf, int ktot, int N)
{
    const int r = blockIdx.y;
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const PrimeConst &c = pc[r % ktot];
    if (!c.fp) return;
    const long o = (long)r * N + n;
    kf[o] = (u64)__double_as_longlong((double)redc(kmont[o], 0, c));
}

void launch_key_fp(const PrimeConst *pc, const u64 *kmont, u64 *kf, int rows, int ktot, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, rows);
    hipLaunchKernelGGL(k_key_fp, g, dim3(256), 0, s, pc, kmont, kf, ktot, N);
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


// ---------------------------------------------------------------- ModRaise
// coefficient n of polynomial p (mod q_0) as a centred integer, reduced mod
// the prime of the output limb
__global__ void k_modraise(const PrimeConst *pc, PolySet out, const u64 *in, LimbMap lm, int N)
{
    const int y = blockIdx.y;
    const int poly = y % out.npoly, limb = y / out.npoly;
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const u64 q0 = pc[0].q, q = pc[lm.prime(limb)].q;
    const u64 v = in[(long)poly * N + n];
    u64 r;
    if (2 * v > q0) {
        const u64 a = (q0 - v) % q;
        r = a ? q - a : 0;
    } else {
        r = v % q;
    }
    out.base[limb * out.lstride + poly * out.pstride + n] = r;
}

void launch_modraise(const PrimeConst *pc, PolySet out, const u64 *in, LimbMap lm, int N, hipStream_t s)
{
    dim3 g((N + 255) / 256, out.nl * out.npoly);
    hipLaunchKernelGGL(k_modraise, g, dim3(256), 0, s, pc, out, in, lm, N);
}

}  // namespace hk
