// Shared declarations between the host runtime and the HIP kernels of the
// RNS-CKKS ring layer (limb-major residues, 64-bit words, primes < 2^61).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hk {

typedef unsigned long long u64;
typedef uint32_t u32;

// Per-prime constants, one entry per prime of the chain [q_0..q_L, p_0..p_{a-1}].
struct PrimeConst {
    u64 q;
    u64 mu;        // floor(2^(2b) / q), Barrett for products < 2^(2b)
    u64 qinv_neg;  // -q^-1 mod 2^64 (Montgomery REDC)
    u64 r1, r1p;   // 2^64 mod q and its Shoup companion
    u64 ninv, ninvp;
    int bits;      // b = bit length of q
    int fp;        // 1: the transforms of this prime run in exact FP64 arithmetic (q < 2^46)
    double qd, qinvd;  // q and 1/q as doubles
    double r32d, r32c; // 2^32 mod q and (2^32 mod q) / q as doubles (FP64 primes)
};

// FP64 twiddle: w and w/q (w < q < 2^46 is exact in a double)
struct alignas(16) TwF {
    double w, c;
};

// Which prime each limb of a polynomial uses: limbs [0, nq) take q_0..q_{nq-1},
// limbs [nq, ...) take the special primes p_0.. (stored at index L1 + i).
struct LimbMap {
    int nq;
    int L1;         // L + 1 = index of p_0 in the prime table
    int q_off = 0;  // limb i < nq uses q_{i + q_off}
    __host__ __device__ int prime(int limb) const { return limb < nq ? limb + q_off : L1 + (limb - nq); }
};

// A strided set of polynomials: polynomial `p`, limb `l` starts at
// base + l * lstride + p * pstride.
struct PolySet {
    u64 *base;
    long lstride;
    long pstride;
    int nl;     // limbs
    int npoly;  // polynomials sharing the limb structure
};

struct NttTables {
    const PrimeConst *pc;  // [nprimes]
    const u64 *fw, *fwp;   // psi^brv(k) and Shoup companions, [nprimes][N]
    const u64 *iw, *iwp;   // psi^-brv(k)
    const TwF *ffw, *fiw;  // the same twiddles as FP64 pairs, [nprimes][N]
    // factors of the second-pass twiddles (the last 8 stages): entry
    // 2^st + (r << s) + u, st = logN - 8 + s, is A(r, s) B(s, u) with
    // A(r, s) = W[2^st + (r << s)] ([nprimes][rows][8]) and
    // B(s, u) = W[2^st + u] / W[2^st] ([nprimes][256] at (1 << s) - 1 + u);
    // forward (fa, fb) and inverse (ia, ib), FP64 pairs
    const TwF *fa, *fb, *ia, *ib;
    int logN;
};

// Optional per-kernel timer: HIP events recorded on the launch stream around
// every launch of one selected kernel, with the launch's algorithmic bytes and
// butterflies/multiply-accumulates.
enum KernelId { KID_NTT_FWD1 = 0, KID_NTT_FWD2, KID_NTT_INV2, KID_NTT_INV1, KID_BCONV, KID_KEYIP, KID_MODUP_KEYIP, KID_COUNT };
struct KernelTimer {
    int target = -1;
    struct Rec {
        hipEvent_t a, b;
        double bytes, ops;
    };
    Rec *recs = nullptr;
    size_t used = 0, cap = 0;
    bool on(int id) const { return id == target; }
    void before(hipStream_t s);
    void after(hipStream_t s, double bytes, double ops);
};

// ------------------------------------------------------------------ launchers
void launch_ntt(const NttTables &t, PolySet ps, LimbMap lm, int skip_lo, int skip_hi, bool inverse,
                hipStream_t s, KernelTimer *tm = nullptr);

// out = a op b elementwise over (limb, poly, coeff); op: 0 add, 1 sub
void launch_addsub(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int op, int N,
                   hipStream_t s);
// out = a * k_l (per-limb scalar residue table ks[limb], Shoup table ksp)
void launch_mul_scalar(const PrimeConst *pc, PolySet out, PolySet a, const u64 *ks, const u64 *ksp,
                       LimbMap lm, int N, hipStream_t s);
// out = k a (kf non-null: per-limb factor k mod q and its Shoup word kfp) with
// component 0 of every ciphertext plus a per-limb constant c[limb] (c
// non-null) or plus the plaintext polynomial p [limb][N] (p non-null); out
// and a are ciphertext sets (polynomial 2 e + component)
void launch_add_c0(const PrimeConst *pc, PolySet out, PolySet a, const u64 *kf, const u64 *kfp, const u64 *c,
                   const u64 *p, LimbMap lm, int N, hipStream_t s);
// tensor (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1), accumulate if acc
void launch_tensor(const PrimeConst *pc, PolySet d, PolySet a, PolySet b, LimbMap lm, int N, bool acc,
                   hipStream_t s);
// out[p] = REDC(sum_k a_k[p] * pt_k), pt in Montgomery form; k < nterms
// a_ptrs: device array of nterms PolySet-equivalent base pointers
void launch_lincomb(const PrimeConst *pc, PolySet out, const u64 *const *a_bases, long a_lstride,
                    long a_pstride, const u64 *const *pt_bases, long pt_lstride, int nterms, LimbMap lm,
                    int N, hipStream_t s);
// automorphism in the NTT domain, out[j] = a[perm_g(j)]
void launch_automorph(PolySet out, PolySet a, u64 g, int logN, hipStream_t s);
// out[j] = [out[j] +] a[perm_g(j)] modulo each limb's prime (lm), plus on
// component 0 (even polynomials) of the Q limbs (< nq) pm[i] c0[perm_g(j)]
// (pm: P mod q_i by prime index, pmp its Shoup words); c0 holds one
// polynomial per pair of a's
void launch_automorph_acc(const PrimeConst *pc, PolySet out, PolySet a, PolySet c0, const u64 *pm, const u64 *pmp,
                          u64 g, int logN, LimbMap lm, int nq, bool accumulate, hipStream_t s);
// inner product of the extended digits with a switching key (NTT +
// Montgomery form): acc_c[t] = sum_j e_j[t] * key_j[c][kt(t)], c = 0, 1, where
// e_j[t] is the input d itself on digit j's own limbs and ext_j[t] elsewhere.
// Galois keys are stored permuted by sigma^-1, so no permutation happens here.
// nl limbs t = i < skip_lo ? i : i + skip_hi - skip_lo (i < nl) are computed.
// Returns -1 (nothing launched) unless 1 <= ndig <= 16.
int launch_keyip(const PrimeConst *pc, u64 *acc, long acc_pstride, long acc_bstride, const u64 *ext,
                 long ext_dstride, long ext_bstride, const u64 *d, long d_ls, long d_bstride, const u64 *key,
                 long key_dstride, long key_cstride, int ndig, int nl, int skip_lo, int skip_hi, int nq, int w,
                 int nb, LimbMap lm, int key_nq_off, int logN, hipStream_t s, KernelTimer *tm = nullptr);
// the double (standard form) copy of a switching key's FP64-prime limbs: rows
// r of N words, limb r mod ktot (prime index), from Montgomery words
void launch_key_fp(const PrimeConst *pc, const u64 *kmont, u64 *kf, int rows, int ktot, int N, hipStream_t s);

// --- fused transforms (ntt.hip)
// inverse transform of src (through sigma_galois if galois > 1) into `work`;
// limb i is multiplied by scale[i] (N^-1 folded in), or by N^-1 if scale is null
void launch_intt_from(const NttTables &t, PolySet work, LimbMap lm, const u64 *src, long src_ls, long src_ps,
                      u64 galois, const u64 *scale, const u64 *scalep, hipStream_t s, KernelTimer *tm = nullptr);
// the inverse transform that starts ModUp: like launch_intt_from with a scale
// table, but a limb on an FP64 prime takes its factor from scalef (value and
// quotient constant) and is stored as the bits of a double in [0, q)
void launch_intt_modup(const NttTables &t, PolySet work, LimbMap lm, const u64 *src, long src_ls, long src_ps,
                       const u64 *scale, const u64 *scalep, const TwF *scalef, hipStream_t s,
                       KernelTimer *tm = nullptr);
// ModUp of every digit of nb ciphertexts at once: ext [nb][ndig][nq+alpha][N] <-
// NTT(BConv(y_digit)) on every limb outside the digit; y [nb][nq][N];
// hatm [ndig][w][nq+alpha] Montgomery form; hatf the same constants in
// standard form as FP64 pairs (used for targets on FP64 primes); bit
// 8 j + k of wide (j < 8: wide[0], else wide[1]) marks source k of digit j as
// a prime of more than 50 bits, the same bit of dbl a source held as the bits
// of a double (written by launch_intt_modup)
void launch_modup(const NttTables &t, u64 *ext, int ndig, int nq, int alpha, int w, int nb, LimbMap lm,
                  const u64 *y, const u64 *hatm, const TwF *hatf, const u64 wide[2], const u64 dbl[2], hipStream_t s,
                  KernelTimer *tm = nullptr);
// the key inner product fused into ModUp's second pass on the limbs [fp_lo, fp_hi)
// of FP64 primes (the other limbs' extended digits are stored as by launch_modup);
// d: limb t of element e at d + t d_ls + e d_es; kf: key words in standard form as
// doubles, digit j component c limb t at kf + j kf_ds + c kf_cs + t N; acc: element e
// component c limb t at acc + e acc_es + c acc_cs + t N; own_int: the own limbs of
// one element outside [fp_lo, fp_hi)
struct ModupKeyipArgs {
    int fp_lo, fp_hi, own_int, nb;
    const u64 *d;
    long d_ls, d_es;
    const double *kf;
    long kf_ds, kf_cs;
    u64 *acc;
    long acc_es, acc_cs;
    int gspan = 8;  // (limb, tile) groups per span of the block order (8: one XCD per group)
};
void launch_modup_keyip(const NttTables &t, u64 *ext, int ndig, int nq, int alpha, int w, int nb, LimbMap lm,
                        const u64 *y, const u64 *hatm, const TwF *hatf, const u64 wide[2], const u64 dbl[2],
                        const ModupKeyipArgs &a, hipStream_t s, KernelTimer *tm = nullptr);
struct OutModdownArgs {
    const u64 *acc;
    long acc_ls, acc_ps;
    const u64 *base;  // element e component c of limb i at base + i bls + e bes + c bcs
    long bls, bes, bcs;
    int mask;  // bit c: add base component c (component 0 through sigma_galois)
    u64 galois;
    u64 *out;
    long ols, ops;
    const u64 *pinv, *pinvp;
    // optional addend (null: none), added unpermuted to both components:
    // element e component c of limb i at add + i als + e aes + c N
    const u64 *add = nullptr;
    long als = 0, aes = 0;
    const TwF *pinvf = nullptr;  // pinv as FP64 pairs (value, value / q_i), read on FP64 primes
};
// ModDown of npoly (= 2 nb) polynomials: out_p = base_p + (acc_p - NTT(BConv_{P->Q}(yP_p))) P^-1,
// tmp [npoly][nq][N], yP [npoly][alpha][N]
void launch_moddown(const NttTables &t, u64 *tmp, int nq, int alpha, int npoly, LimbMap lm, const u64 *yP,
                    const u64 *hatm, long hat_ks, const OutModdownArgs &a, hipStream_t s, KernelTimer *tm = nullptr);
// ModDown followed by the rescale by q_l, for a relinearisation (no automorphism, both
// base components): limbs i < l of out = (base_i [+ cadd_i on component 0] + KS_i) k q_l^-1,
// where KS is the ModDown of acc; `last` holds limb l of that sum in coefficient form
struct OutModdownRescaleArgs {
    const u64 *acc;
    long acc_ls, acc_ps;
    const u64 *base;
    long bls, bes, bcs;
    u64 *out;
    long ols, ops;
    const u64 *pinv, *pinvp;
    const TwF *pinvf;
    const u64 *inv, *invp;  // k q_l^-1 mod q_i and Shoup words
    const TwF *invf;
    const u64 *cadd;        // null, or per limb the constant c / inv (mod q_i) for component 0
};
void launch_moddown_rescale(const NttTables &t, u64 *tmp, int l, int alpha, int npoly, const u64 *yP,
                            const u64 *hatm, long hat_ks, const u64 *last, u64 ql, const u64 *pm, const u64 *pmp,
                            const TwF *pmf, const OutModdownRescaleArgs &a, int L1, hipStream_t s,
                            KernelTimer *tm = nullptr);
// rescale by q_l of npoly polynomials: out_i = (in_i pm_i [+ cadd_i on even polynomials] - NTT_i([last + h] - h)) inv_i,
// inv_i = k q_l^-1 mod q_i for an integer factor k (invf: as FP64 pairs (value, value / q_i), read on FP64
// primes); pm (Shoup words pmp) a per-limb factor, or null for 1
void launch_rescale_ntt(const NttTables &t, u64 *tmp, int l, int npoly, const u64 *last, u64 ql, const u64 *in,
                        long in_ls, long in_ps, u64 *out, long out_ls, long out_ps, const u64 *inv, const u64 *invp,
                        const TwF *invf, const u64 *pm, const u64 *pmp, const u64 *cadd, int L1, hipStream_t s,
                        KernelTimer *tm = nullptr);
// copy limbs
void launch_copy(PolySet out, PolySet in, int N, hipStream_t s);
// ModRaise: polynomial p of `in` ([npoly][N], coefficients mod q_0) read as
// centred integers and reduced mod the prime of every limb of out
void launch_modraise(const PrimeConst *pc, PolySet out, const u64 *in, LimbMap lm, int N, hipStream_t s);
// pointwise product out = a * b (single polynomials, Barrett)
void launch_pmul(const PrimeConst *pc, PolySet out, PolySet a, PolySet b, LimbMap lm, int N, hipStream_t s);
// switching-key body b = e - a s + pfac s' (NTT domain); b and a leave in Montgomery form
void launch_keygen_b(const PrimeConst *pc, u64 *b, const u64 *a, const u64 *s, const u64 *e,
                     const u64 *sp, const u64 *pfac, int ntot, int N, hipStream_t st);
void launch_to_montgomery(const PrimeConst *pc, u64 *x, long lstride, int nl, LimbMap lm, int N,
                          int npoly, long pstride, hipStream_t s);
// decryption on limb 0: m = c0 + c1 * s (NTT domain)
void launch_decrypt0(const PrimeConst *pc, u64 *m, const u64 *c0, const u64 *c1, const u64 *s, int N,
                     hipStream_t st);
// encryption: c0 = -a s + e + m (NTT domain), per limb
void launch_encrypt(const PrimeConst *pc, u64 *c0, const u64 *a, const u64 *s, const u64 *em, long c_lstride,
                    int nl, int N, hipStream_t st);

}  // namespace hk
