// Negacyclic NTT kernels for gfx950 and the key-switch / rescale pipelines
// fused into them.
//
// The transform is Cooley-Tukey with the psi twist merged into the twiddles
// (bit-reversed psi powers): natural-order input, bit-reversed output; the
// inverse is Gentleman-Sande.  N = R * C with C = 2^min(logN, 8).  Pass 1 runs
// the first log R stages on columns (elements c, c+C, c+2C, ...) with a
// 4096-word tile of at least 16 adjacent columns per workgroup; pass 2 runs
// the last log C stages on contiguous rows of C words, 8 rows per workgroup.
// Inside a pass every thread holds a radix-8 unit (three stages) in
// registers; units are exchanged through LDS between phases.
//
// Each limb takes one of two arithmetic paths, chosen per workgroup by its
// prime: primes below 2^46 use exact FP64 arithmetic (full-rate FMA, values
// kept as signed integers in doubles, no reduction inside a forward
// transform); wider primes use Harvey's lazy butterflies on 64-bit words
// (forward values in [0, 4q), inverse values in [0, 2q)).
//
// The first load and the last store of each transform go through policy
// objects, so neighbouring ring steps run inside the transform instead of as
// separate passes over HBM:
//   * fast basis conversion (ModUp of every key-switch digit, ModDown from P)
//     is computed on the pass-1 load of the forward transform;
//   * the rescale input ([c_l + h]_{q_l} - h) mod q_i is formed on that load,
//     and (c_i - t_i) q_l^-1 on the pass-2 store;
//   * the ModDown tail base + (acc - conv) P^-1 runs on the pass-2 store;
//   * inverse transforms read their input from another buffer (optionally
//     through a Galois permutation) and fold a per-limb constant into N^-1.
#include "dev.hpp"
#include <type_traits>

#include "modarith.hpp"

namespace hk {

template <int LOGN>
struct NttGeo {
    static constexpr int LC = LOGN < 8 ? LOGN : 8;
    static constexpr int LR = LOGN - LC;
    // pass-1 tile: 2^12 words, so a tile row spans at least 16 columns (one
    // 128-byte line); pass-2 tile: 2^11 words of whole rows
    static constexpr int LTC = (12 - LR) < LC ? (12 - LR) : LC;
    static constexpr int LRB = (11 - LC) < LR ? (11 - LC) : LR;
};

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

__device__ __forceinline__ u64 reduce4(u64 v, u64 q)
{
    v = v >= 2 * q ? v - 2 * q : v;
    return v >= q ? v - q : v;
}

// ------------------------------------------------------------------ policies
// Context of one block: working polynomial pointer, limb, polynomial, prime.
struct Blk {
    u64 *a;
    int limb, poly;
    const PrimeConst *pc;
    int logN;
    int tid;  // threadIdx.x, for OutLds only (see OpaqueTid)
};

// Every policy states the words it reads per coefficient position over a
// launch of npoly polynomials x nl limbs (read_words for inputs, extra_words
// for outputs), for the algorithmic byte count of the kernel timer.
struct InWork {
    __device__ u64 load(const Blk &b, long g) const { return b.a[g]; }
    double read_words(int npoly, int nl) const { return (double)npoly * nl; }
};

// read the same (limb, poly) of another set, through sigma_galois if galois > 1
struct InSrc {
    const u64 *base;
    long ls, ps;
    u64 galois;
    __device__ u64 load(const Blk &b, long g) const
    {
        long gg = galois > 1 ? (long)auto_src((u32)g, galois, b.logN) : g;
        return base[b.limb * ls + b.poly * ps + gg];
    }
    double read_words(int npoly, int nl) const { return (double)npoly * nl; }
};

// fast basis conversion: sum_k y_k * hat(k, target) with y in coefficient form
// (already multiplied by the inverse hat constants), hat in Montgomery form
struct InBconv {
    // polynomial p = e ndig + j (batch element e, digit j): sources at
    // src + e src_bs + j src_ps, limb stride N; hat(k, t) at hatm[j hat_ps + k hat_ks + t]
    const u64 *src;
    long src_bs, src_ps;
    const u64 *hatm;
    long hat_ps, hat_ks;
    int ndig;
    int ns_fixed;       // > 0: every polynomial has ns_fixed sources
    int w, nq;          // else digit j has min(w, nq - j w) sources
    const TwF *hatf;    // non-null: FP64 pairs (hat, hat / q_t), same indexing, for FP64 targets
    u64 wide[2];        // bit 8 j + k: source k of digit j is a prime above 2^50
    u64 dbl[2];         // bit 8 j + k: source k of digit j holds the bits of a double (an FP64 prime's residue)
    __device__ u64 bits(const u64 *m, int j) const { return (j < 8 ? m[0] >> (8 * j) : m[1] >> (8 * (j - 8))) & 0xff; }
    __device__ int nsrc(int j) const { return ns_fixed > 0 ? ns_fixed : min(w, nq - j * w); }
    // each source limb is read once per launch: the ndig digits of a batch
    // element together hold its nq limbs
    double read_words(int npoly, int) const
    {
        return ns_fixed > 0 ? (double)npoly * ns_fixed : (double)(npoly / ndig) * nq;
    }
    __device__ u64 load(const Blk &b, long g) const
    {
        const int e = b.poly / ndig, j = b.poly - e * ndig;
        const int ns = nsrc(j);
        const long N = 1l << b.logN;
        const u64 *s = src + e * src_bs + j * src_ps + g;
        const u64 *h = hatm + j * hat_ps + b.limb;
        const u64 dj = bits(dbl, j);
        u64 lo = 0, hi = 0;
        for (int k = 0; k < ns; k++) mac(lo, hi, dj >> k & 1 ? d2u_exact(s[k * N]) : s[k * N], h[k * hat_ks]);
        return redc(lo, hi, *b.pc);
    }
    // M positions at once, sources outermost: M independent loads in flight
    // per source instead of one dependent chain per position
    template <int M>
    __device__ void load_many(const Blk &b, const long *g, u64 *x) const
    {
        const int e = b.poly / ndig, j = b.poly - e * ndig;
        const int ns = nsrc(j);
        const long N = 1l << b.logN;
        const u64 *s = src + e * src_bs + j * src_ps;
        const u64 *h = hatm + j * hat_ps + b.limb;
        const u64 dj = bits(dbl, j);
        u64 lo[M], hi[M];
#pragma unroll
        for (int m = 0; m < M; m++) lo[m] = hi[m] = 0;
#pragma unroll 1
        for (int k = 0; k < ns; k++) {
            const u64 hk = h[k * hat_ks];
            u64 y[M];
#pragma unroll
            for (int m = 0; m < M; m++) y[m] = s[k * N + g[m]];
            if (dj >> k & 1) {
#pragma unroll
                for (int m = 0; m < M; m++) y[m] = d2u_exact(y[m]);
            }
#pragma unroll
            for (int m = 0; m < M; m++) mac(lo[m], hi[m], y[m], hk);
        }
#pragma unroll
        for (int m = 0; m < M; m++) x[m] = redc(lo[m], hi[m], *b.pc);
    }
    // the same sums for a target on an FP64 prime, reduced to |x| <= q/2 + 1:
    // each term is one exact FP64 modular product; a source word above 2^50
    // is first folded to (y >> 32)(2^32 mod q) + (y mod 2^32)
    template <int M>
    __device__ void load_many_d(const Blk &b, const long *g, double *x) const
    {
        if (!hatf) {
            u64 v[M];
            load_many<M>(b, g, v);
#pragma unroll
            for (int m = 0; m < M; m++) x[m] = u2d(v[m]);
            return;
        }
        const int e = b.poly / ndig, j = b.poly - e * ndig;
        const int ns = nsrc(j);
        const long N = 1l << b.logN;
        const u64 *s = src + e * src_bs + j * src_ps;
        const TwF *h = hatf + j * hat_ps + b.limb;
        const double q = b.pc->qd;
        const u64 wj = bits(wide, j), dj = bits(dbl, j);
        double acc[M];
#pragma unroll
        for (int m = 0; m < M; m++) acc[m] = 0.0;
#pragma unroll 1
        for (int k = 0; k < ns; k++) {
            const TwF t = h[k * hat_ks];
            u64 y[M];
#pragma unroll
            for (int m = 0; m < M; m++) y[m] = s[k * N + g[m]];
            if (wj >> k & 1) {
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const double yd = mulm_fp(u2d(y[m] >> 32), b.pc->r32d, b.pc->r32c, q) + u2d(y[m] & 0xffffffffull);
                    acc[m] += mulm_fp(yd, t.w, t.c, q);
                }
            } else if (dj >> k & 1) {
#pragma unroll
                for (int m = 0; m < M; m++) acc[m] += mulm_fp(__longlong_as_double((long long)y[m]), t.w, t.c, q);
            } else {
#pragma unroll
                for (int m = 0; m < M; m++) acc[m] += mulm_fp(u2d(y[m]), t.w, t.c, q);
            }
        }
        const double qi = b.pc->qinvd;
#pragma unroll
        for (int m = 0; m < M; m++) x[m] = __fma_rn(-rint(acc[m] * qi), q, acc[m]);
    }
};

// rescale input ([c_l + h]_{q_l} - h) mod q_i from the dropped limb c_l
struct InRescale {
    const u64 *last;  // polynomial p at last + p * last_ps (coefficient form)
    long last_ps;
    u64 ql;
    double qld, hd;   // q_l and floor(q_l / 2) as doubles, when q_l < 2^52 (else qld = 0)
    __device__ u64 load(const Blk &b, long g) const
    {
        const u64 h = ql >> 1;
        u64 r = last[b.poly * last_ps + g] + h;
        r = r >= ql ? r - ql : r;
        return subm(reduce64(r, *b.pc), reduce64(h, *b.pc), b.pc->q);
    }
    // for an FP64 target: [c_l + h]_{q_l} - h is an integer of magnitude at
    // most q_l / 2, formed exactly in FP64 and reduced to |x| <= q/2 + 1 (the
    // same residue as load(), in the balanced range the transform accepts)
    __device__ double load_d(const Blk &b, long g) const
    {
        if (qld == 0.0) return u2d(load(b, g));
        double t = u2d(last[b.poly * last_ps + g]) + hd;
        t = t >= qld ? t - qld : t;
        const double v = t - hd;
        return __fma_rn(-rint(v * b.pc->qinvd), b.pc->qd, v);
    }
    double read_words(int npoly, int) const { return (double)npoly; }  // the dropped limb, shared by all limbs
    // M positions at once: every word is requested before the first is used,
    // so the M reads are in flight together
    template <int M>
    __device__ void load_many(const Blk &b, const long *g, u64 *x) const
    {
        const u64 *src = last + b.poly * last_ps;
#pragma unroll
        for (int m = 0; m < M; m++) x[m] = src[g[m]];
        const u64 h = ql >> 1, hq = reduce64(h, *b.pc);
#pragma unroll
        for (int m = 0; m < M; m++) {
            u64 r = x[m] + h;
            r = r >= ql ? r - ql : r;
            x[m] = subm(reduce64(r, *b.pc), hq, b.pc->q);
        }
    }
    template <int M>
    __device__ void load_many_d(const Blk &b, const long *g, double *x) const
    {
        const u64 *src = last + b.poly * last_ps;
        u64 raw[M];
#pragma unroll
        for (int m = 0; m < M; m++) raw[m] = src[g[m]];
        if (qld == 0.0) {
            const u64 h = ql >> 1, hq = reduce64(h, *b.pc);
#pragma unroll
            for (int m = 0; m < M; m++) {
                u64 r = raw[m] + h;
                r = r >= ql ? r - ql : r;
                x[m] = u2d(subm(reduce64(r, *b.pc), hq, b.pc->q));
            }
            return;
        }
#pragma unroll
        for (int m = 0; m < M; m++) {
            double t = u2d(raw[m]) + hd;
            t = t >= qld ? t - qld : t;
            const double v = t - hd;
            x[m] = __fma_rn(-rint(v * b.pc->qinvd), b.pc->qd, v);
        }
    }
};

// Output policies.  NPRE > 0: the policy reads NPRE further words per output
// position; the kernel loads them with fetch() before the first phase, so
// they are in flight during the butterflies, and hands them to store().
enum { OW_LAZY = 0, OW_REDUCE = 1, OW_SCALE_N = 2 };
template <int MODE>
struct OutWork {
    static constexpr int NPRE = 0;
    double extra_words(int, int) const { return 0; }
    __device__ void fetch(const Blk &, long, u64 *) const {}
    __device__ void store(const Blk &b, long g, u64 v, const u64 *) const
    {
        const u64 q = b.pc->q;
        if (MODE == OW_REDUCE) v = reduce4(v, q);
        if (MODE == OW_SCALE_N) {
            v = shoup_lazy(v, b.pc->ninv, b.pc->ninvp, q);
            v = v >= q ? v - q : v;
        }
        b.a[g] = v;
    }
};

// inverse transform, last store: multiply by a per-limb constant (N^-1 folded in)
struct OutScaleTab {
    const u64 *s, *sp;
    static constexpr int NPRE = 0;
    double extra_words(int, int) const { return 0; }
    __device__ void fetch(const Blk &, long, u64 *) const {}
    __device__ void store(const Blk &b, long g, u64 v, const u64 *) const
    {
        const u64 q = b.pc->q;
        v = shoup_lazy(v, s[b.limb], sp[b.limb], q);
        b.a[g] = v >= q ? v - q : v;
    }
};

// inverse transform, last store of the basis-conversion sources of ModUp: limb
// i times scale[i] (N^-1 folded in); on an FP64 prime the product is taken in
// FP64 (sf: the factor and its quotient constant), reduced to [0, q) and stored
// as the bits of the double, which the conversion reads without converting
struct OutScaleTabFp {
    const u64 *s, *sp;
    const TwF *sf;
    static constexpr int NPRE = 0;
    double extra_words(int, int) const { return 0; }
    __device__ void fetch(const Blk &, long, u64 *) const {}
    __device__ void store(const Blk &b, long g, u64 v, const u64 *) const
    {
        const u64 q = b.pc->q;
        v = shoup_lazy(v, s[b.limb], sp[b.limb], q);
        b.a[g] = v >= q ? v - q : v;
    }
    __device__ void store_d(const Blk &b, long g, double v) const
    {
        const double q = b.pc->qd;
        const TwF f = sf[b.limb];
        double r = mulm_fp(v, f.w, f.c, q);
        r = r < 0.0 ? r + q : r;
        b.a[g] = (u64)__double_as_longlong(r);
    }
};

// rescale tail: out = (in - t) * q_l^-1
// inv holds k q_l^-1 mod q_i for an integer factor k (1 for a plain rescale);
// pm, if set, a per-limb factor the input is multiplied by when it is fetched
// (Shoup words pmp); cadd, if set, holds per limb a word added to component 0 (polynomial
// p = 2 e + c, c = 0) of every ciphertext before the subtraction: a constant
// c lands in the output as cadd = c / inv (mod q_i)
struct OutRescaleFin {
    const u64 *in;
    long ls, ps;
    u64 *out;
    long ols, ops;
    const u64 *inv, *invp;
    const TwF *invf;  // inv as FP64 pairs (value, value / q) for FP64 primes
    const u64 *pm, *pmp;
    const u64 *cadd;
    static constexpr int NPRE = 1;
    double extra_words(int npoly, int nl) const { return (double)npoly * nl; }
    // the word is only requested here (nothing uses it yet, so every prefetch
    // of the block is in flight together); prepare() applies the factor and
    // the constant once the last phase begins, before the block's first store
    __device__ void fetch(const Blk &b, long g, u64 *pre) const { pre[0] = in[b.limb * ls + b.poly * ps + g]; }
    __device__ void prepare(const Blk &b, u64 *pre) const
    {
        u64 x = pre[0];
        if (pm) x = shoup(x, pm[b.limb], pmp[b.limb], b.pc->q);
        pre[0] = cadd && (b.poly & 1) == 0 ? addm(x, cadd[b.limb], b.pc->q) : x;
    }
    __device__ void store(const Blk &b, long g, u64 v, const u64 *pre) const
    {
        const u64 q = b.pc->q;
        v = reduce4(v, q);
        out[b.limb * ols + b.poly * ops + g] = shoup(subm(pre[0], v, q), inv[b.limb], invp[b.limb], q);
    }
    // FP64 prime: v is the transform's unreduced output (|v| <= 17q), the
    // product is one exact FP64 modular product within 3q/4 of zero
    __device__ void store_d(const Blk &b, long g, double v, const u64 *pre) const
    {
        const double q = b.pc->qd;
        const TwF f = invf[b.limb];
        double r = mulm_fp(u2d(pre[0]) - v, f.w, f.c, q);
        r = r < 0.0 ? r + q : r;
        out[b.limb * ols + b.poly * ops + g] = d2u_exact((u64)__double_as_longlong(r));
    }
};

// ModDown tail: out_p = base_p + (acc_p - conv_p) * P^-1 [+ add_p] for
// polynomial p = 2 e + c; acc and base component 0 read through sigma_galois,
// the optional addend unpermuted (rotate-and-add in one pass)
struct OutModdownFin {
    const u64 *acc;
    long acc_ls, acc_ps;
    const u64 *base;
    long bls, bes, bcs;
    int mask;
    u64 galois;
    u64 *out;
    long ols, ops;
    const u64 *pinv, *pinvp;
    const u64 *add;
    long als, aes;
    const TwF *pinvf;  // pinv as FP64 pairs (value, value / q) for FP64 primes
    static constexpr int NPRE = 3;
    double extra_words(int npoly, int nl) const
    {
        return (double)npoly * nl * (add ? 2.0 : 1.0) +
               (double)(npoly / 2) * nl * ((mask & 1) + (mask >> 1 & 1));
    }
    __device__ void fetch(const Blk &b, long g, u64 *pre) const
    {
        const long gp = galois > 1 ? (long)auto_src((u32)g, galois, b.logN) : g;
        pre[0] = acc[b.limb * acc_ls + b.poly * acc_ps + gp];
        const int e = b.poly >> 1, c = b.poly & 1;
        pre[1] = (mask >> c & 1) ? base[b.limb * bls + e * bes + c * bcs + (c == 0 ? gp : g)] : 0;
        pre[2] = add ? add[b.limb * als + e * aes + ((long)c << b.logN) + g] : 0;
    }
    __device__ void store(const Blk &b, long g, u64 v, const u64 *pre) const
    {
        const u64 q = b.pc->q;
        v = reduce4(v, q);
        u64 r = shoup(subm(pre[0], v, q), pinv[b.limb], pinvp[b.limb], q);
        if (mask >> (b.poly & 1) & 1) r = addm(r, pre[1], q);
        if (add) r = addm(r, pre[2], q);
        out[b.limb * ols + b.poly * ops + g] = r;
    }
    // FP64 prime: (acc - v) P^-1 as one exact FP64 modular product (|v| <= 17q),
    // plus the base and addend words (each below q), then reduced to [0, q)
    __device__ void store_d(const Blk &b, long g, double v, const u64 *pre) const
    {
        const double q = b.pc->qd;
        const TwF f = pinvf[b.limb];
        double r = mulm_fp(u2d(pre[0]) - v, f.w, f.c, q);
        if (mask >> (b.poly & 1) & 1) r += u2d(pre[1]);
        if (add) r += u2d(pre[2]);
        out[b.limb * ols + b.poly * ops + g] = d2u_mod(r, q, b.pc->qinvd);
    }
};

// ModDown's basis conversion with the rescale that follows a relinearisation
// folded in.  Besides the conversion of the P limbs (InBconv), each output word
// gets P_i r, where r = ([c_l + h]_{q_l} - h) mod q_i is the rescale's input
// word (limb l of the key-switched ciphertext in coefficient form, h =
// floor(q_l / 2)) and P_i = P mod q_i.  The transform is linear, so
// NTT(conv + P_i r) P^-1 = NTT(conv) P^-1 + NTT(r): the ModDown tail below then
// forms c_i - NTT(r), which the rescale multiplies by q_l^-1.
struct InBconvRs : InBconv {
    const u64 *last;  // polynomial p at last + p last_ps
    long last_ps;
    u64 ql;
    double qld, hd;       // q_l and floor(q_l / 2) as doubles, when q_l < 2^52 (else qld = 0)
    const u64 *pm, *pmp;  // P mod q_i and Shoup words
    const TwF *pmf;       // P mod q_i as FP64 pairs (value, value / q_i)
    double read_words(int npoly, int nl) const { return InBconv::read_words(npoly, nl) + (double)npoly; }
    template <int M>
    __device__ void load_many(const Blk &b, const long *g, u64 *x) const
    {
        const u64 *src = last + b.poly * last_ps;
        u64 rw[M];
#pragma unroll
        for (int m = 0; m < M; m++) rw[m] = src[g[m]];
        InBconv::template load_many<M>(b, g, x);  // below q
        const u64 q = b.pc->q, h = ql >> 1, hq = reduce64(h, *b.pc);
        const u64 w = pm[b.limb], wp = pmp[b.limb];
#pragma unroll
        for (int m = 0; m < M; m++) {
            u64 r = rw[m] + h;
            r = r >= ql ? r - ql : r;
            r = subm(reduce64(r, *b.pc), hq, q);
            x[m] = addm(x[m], shoup(r, w, wp, q), q);
        }
    }
    // FP64 target: the rescale term in exact FP64 arithmetic (r within q/2 + 1
    // of zero, P_i r one exact product within 3q/4), added to the conversion
    // word (below q): within 4q, as the transform accepts
    template <int M>
    __device__ void load_many_d(const Blk &b, const long *g, double *x) const
    {
        if (qld == 0.0) {
            u64 v[M];
            load_many<M>(b, g, v);
#pragma unroll
            for (int m = 0; m < M; m++) x[m] = u2d(v[m]);
            return;
        }
        const u64 *src = last + b.poly * last_ps;
        u64 rw[M], v[M];
#pragma unroll
        for (int m = 0; m < M; m++) rw[m] = src[g[m]];
        InBconv::template load_many<M>(b, g, v);
        const double q = b.pc->qd, qi = b.pc->qinvd;
        const TwF f = pmf[b.limb];
#pragma unroll
        for (int m = 0; m < M; m++) {
            double t = u2d(rw[m]) + hd;
            t = t >= qld ? t - qld : t;
            const double r = t - hd;
            x[m] = u2d(v[m]) + mulm_fp(__fma_rn(-rint(r * qi), q, r), f.w, f.c, q);
        }
    }
};

// The tail of that ModDown (no automorphism, both base components): limb i < l
// of the result is (base_i [+ cadd_i on component 0] + (acc_i - v) P^-1) inv_i
// with inv_i = k q_l^-1 mod q_i, v the transform of InBconvRs's words: the
// residues of ModDown followed by the rescale, computed in one pass
struct OutModdownRescaleFin {
    const u64 *acc;
    long acc_ls, acc_ps;
    const u64 *base;
    long bls, bes, bcs;
    u64 *out;
    long ols, ops;
    const u64 *pinv, *pinvp;
    const TwF *pinvf;
    const u64 *inv, *invp;
    const TwF *invf;
    const u64 *cadd;
    static constexpr int NPRE = 2;
    double extra_words(int npoly, int nl) const { return 2.0 * npoly * nl; }
    __device__ void fetch(const Blk &b, long g, u64 *pre) const
    {
        pre[0] = acc[b.limb * acc_ls + b.poly * acc_ps + g];
        pre[1] = base[b.limb * bls + (b.poly >> 1) * bes + (b.poly & 1) * bcs + g];
    }
    __device__ void prepare(const Blk &b, u64 *pre) const
    {
        if (cadd && (b.poly & 1) == 0) pre[1] = addm(pre[1], cadd[b.limb], b.pc->q);
    }
    __device__ void store(const Blk &b, long g, u64 v, const u64 *pre) const
    {
        const u64 q = b.pc->q;
        v = reduce4(v, q);
        const u64 r = addm(shoup(subm(pre[0], v, q), pinv[b.limb], pinvp[b.limb], q), pre[1], q);
        out[b.limb * ols + b.poly * ops + g] = shoup(r, inv[b.limb], invp[b.limb], q);
    }
    // FP64 prime: (acc - v) P^-1 within 3q/4 of zero plus the base word below
    // q, times inv as a second exact product, brought to [0, q)
    __device__ void store_d(const Blk &b, long g, double v, const u64 *pre) const
    {
        const double q = b.pc->qd;
        const TwF f = pinvf[b.limb], s = invf[b.limb];
        const double r = mulm_fp(u2d(pre[0]) - v, f.w, f.c, q) + u2d(pre[1]);
        double o = mulm_fp(r, s.w, s.c, q);
        o = o < 0.0 ? o + q : o;
        out[b.limb * ols + b.poly * ops + g] = d2u_exact((u64)__double_as_longlong(o));
    }
};

// last phase of a second pass leaving the transformed tile in LDS (FP64
// path): position g of the tile's rows goes to the word the row pass itself
// uses for it (row bits 4..6 of the word index XORed into bits 0..3)
struct OutLds {
    double *sh;
    int mask;  // tile words - 1
    static constexpr int NPRE = 0;
    double extra_words(int, int) const { return 0; }
    __device__ void fetch(const Blk &, long, u64 *) const {}
    __device__ void store(const Blk &, long, u64, const u64 *) const {}
    __device__ static int word(int pos)  // pos: row r of the tile, word p: r 256 + p
    {
        const int p = pos & 255;
        return (pos & ~255) + (p ^ (((p >> 4) & 1) | (((p >> 5) & 1) * 6) | (((p >> 6) & 1) << 3)));
    }
    __device__ void store_d(const Blk &, long g, double v) const { sh[word((int)g & mask)] = v; }
};
// the transforms of a kernel that runs several in a loop (OutLds) index with
// a per-iteration copy of threadIdx.x, so their addresses are recomputed per
// transform instead of all being hoisted out of the loop and kept live
template <class OUT> struct OpaqueTid { static constexpr bool value = false; };
template <> struct OpaqueTid<OutLds> { static constexpr bool value = true; };

// between the two passes of one transform: lazy u64 words, or the raw
// balanced doubles of the FP64 path (the next pass of the same prime reads them)
struct InMid {
    __device__ u64 load(const Blk &b, long g) const { return b.a[g]; }
    double read_words(int npoly, int nl) const { return (double)npoly * nl; }
    __device__ double load_d(const Blk &b, long g) const { return __longlong_as_double((long long)b.a[g]); }
};
struct OutMid {
    static constexpr int NPRE = 0;
    double extra_words(int, int) const { return 0; }
    __device__ void fetch(const Blk &, long, u64 *) const {}
    __device__ void store(const Blk &b, long g, u64 v, const u64 *) const { b.a[g] = v; }
    __device__ void store_d(const Blk &b, long g, double v) const { b.a[g] = (u64)__double_as_longlong(v); }
};

template <class IN>
__device__ __forceinline__ double load_fp(const IN &in, const Blk &b, long g)
{
    if constexpr (std::is_same<IN, InMid>::value || std::is_same<IN, InRescale>::value) return in.load_d(b, g);
    else return u2d(in.load(b, g));  // every other input policy yields words below 4q
}

// an output policy with prepare() transforms its prefetched words in place
// when the last phase begins
template <class T, class = void>
struct HasPrepare : std::false_type {};
template <class T>
struct HasPrepare<T, std::void_t<decltype(&T::prepare)>> : std::true_type {};
template <class OUT, class PB>
__device__ __forceinline__ void prepare_pre(const OUT &out, const Blk &bk, PB &pre)
{
    if constexpr (HasPrepare<OUT>::value) {
        constexpr int n = sizeof(pre.v) / sizeof(pre.v[0]);
#pragma unroll
        for (int i = 0; i < n; i++) out.prepare(bk, pre.v[i]);
    }
}

template <class OUT>
__device__ __forceinline__ void store_fp(const OUT &out, const Blk &b, long g, double v, u64 *pre)
{
    if constexpr (std::is_same<OUT, OutMid>::value || std::is_same<OUT, OutScaleTabFp>::value) out.store_d(b, g, v);
    else if constexpr (std::is_same<OUT, OutLds>::value) out.store_d(b, g, v);
    else if constexpr (std::is_same<OUT, OutRescaleFin>::value || std::is_same<OUT, OutModdownFin>::value ||
                       std::is_same<OUT, OutModdownRescaleFin>::value)
        out.store_d(b, g, v, pre);
    else out.store(b, g, d2u_mod(v, b.pc->qd, b.pc->qinvd), pre);
}

// ----------------------------------------------------------------- phases
// One phase of R stages (min distance 2^LS positions) over a tile of
// 2^LP positions x 2^LL lines.  PASS 1: positions are rows, lines columns;
// PASS 2: positions are words of a row, lines rows.  Unit u of the phase owns
// the 2^R positions p0 + k 2^LS of one line.
template <int LOGN, int PASS, int R, int LS>
struct PhaseIdx {
    typedef NttGeo<LOGN> G;
    static constexpr int LP = PASS == 1 ? G::LR : G::LC;
    static constexpr int LL = PASS == 1 ? G::LTC : G::LRB;
    static constexpr int LU = LP - R + LL;
    static constexpr int LHI = LP - LS - R;
    static constexpr int LG = PASS == 1 ? LS + G::LC : LS;  // log2 of the word distance 2^LS positions span
    static constexpr int ITERS = ((1 << LU) + 255) / 256;
    int p0, line;
    long blk;
    // false if unit it * 256 + threadIdx.x does not exist
    __device__ __forceinline__ bool set(int it, long b) { return set(it, b, (int)threadIdx.x); }
    __device__ __forceinline__ bool set(int it, long b, int tid)
    {
        const int u = it * 256 + tid;
        if ((1 << LU) % 256 != 0 && u >= (1 << LU)) return false;
        int lo, hi;
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
        p0 = (hi << (LS + R)) | lo;
        blk = b;
        return true;
    }
    __device__ __forceinline__ long gidx(int k) const
    {
        // positions are below N <= 2^16: 32-bit arithmetic
        const int p = p0 + (k << LS), b = (int)blk;
        return (long)(unsigned)(PASS == 1 ? (p << G::LC) + (b << G::LTC) + line : (((b << G::LRB) + line) << G::LC) + p);
    }
    // LDS word of position k.  Pass 2 keeps whole 256-word rows and XORs row
    // bits 4..6 into bits 0..3 (bit 4 -> 0, bit 5 -> 1 and 2, bit 6 -> 3), so
    // the phases' word strides 1, 4 and 32 all spread 16 consecutive lanes
    // over distinct banks; pass-1 lanes already read 16 consecutive words
    __device__ __forceinline__ int lidx(int k) const
    {
        const int p = p0 + (k << LS);
        if (PASS == 1) return (p << LL) + line;
        if constexpr (LP == 8) return (line << LP) + (p ^ (((p >> 4) & 1) | (((p >> 5) & 1) * 6) | (((p >> 6) & 1) << 3)));
        return (line << LP) + p;
    }
    // the twiddle of the stage-h pair (k, k + 2^h) is entry
    // (N + gidx(k)) >> (LG + h + 1); bits [LG, LG + R) of gidx(0) are clear,
    // so that is tw0(h) + (k >> (h + 1))
    __device__ __forceinline__ long tw0(int h) const
    {
        return (long)(((1u << LOGN) + (unsigned)gidx(0)) >> (LG + h + 1));
    }
};

// NPRE words per position of the last phase, loaded before the first phase
template <int NPRE, int N>
struct PreBuf {
    u64 v[N][NPRE];
};
template <int N>
struct PreBuf<0, N> {
    u64 v[1][1];
};

template <int LOGN, int PASS, bool FWD, int R, int LS, bool FIRST, bool LAST, class IN, class OUT, class PB>
__device__ __forceinline__ void ntt_phase(u64 *sh, const Blk &bk, long blk, const u64 *w, const u64 *wp,
                                          const IN &in, const OUT &out, PB &pre)
{
    typedef PhaseIdx<LOGN, PASS, R, LS> I;
    const u64 q = bk.pc->q, q2 = 2 * q;
    if constexpr (LAST) prepare_pre(out, bk, pre);
#pragma unroll
    for (int it = 0; it < I::ITERS; it++) {
        I ix;
        if (!(OpaqueTid<OUT>::value ? ix.set(it, blk, bk.tid) : ix.set(it, blk))) break;
        u64 x[1 << R];
        if constexpr (FIRST && (std::is_same<IN, InBconv>::value || std::is_same<IN, InRescale>::value ||
                      std::is_same<IN, InBconvRs>::value)) {
            long g[1 << R];
#pragma unroll
            for (int k = 0; k < (1 << R); k++) g[k] = ix.gidx(k);
            in.template load_many<(1 << R)>(bk, g, x);
        } else {
#pragma unroll
            for (int k = 0; k < (1 << R); k++) x[k] = FIRST ? in.load(bk, ix.gidx(k)) : sh[ix.lidx(k)];
        }
        if (FWD) {
#pragma unroll
            for (int h = R - 1; h >= 0; h--) {
                const long ib = ix.tw0(h);
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = ib + (k >> (h + 1));
                    ct_bfly(x[k], x[k + (1 << h)], w[idx], wp[idx], q, q2);
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < R; h++) {
                const long ib = ix.tw0(h);
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = ib + (k >> (h + 1));
                    gs_bfly(x[k], x[k + (1 << h)], w[idx], wp[idx], q, q2);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < (1 << R); k++) {
            if (LAST) out.store(bk, ix.gidx(k), x[k], pre.v[LAST ? (it << R) + k : 0]);
            else sh[ix.lidx(k)] = x[k];
        }
    }
}

// The same phase on the FP64 path (primes below 2^46).  Forward: no reduction
// inside the transform; starting below 4q, sixteen stages that each add at
// most 3q/4 keep every value within 16q <= 2^50.  Inverse: the sum of each
// butterfly is reduced to |s| <= q/2 + 1, the difference stays within 8q.
// Second-pass twiddle of stage s' = LC-1-LS-h from the block's factor tables
// in LDS (shB: B(s', u) at (1 << s') - 1 + u; shA: A(line, s') at 8 line + s'):
// W = A B mod q up to sign (|W| <= 3q/4), with its quotient constant W / q.
__device__ __forceinline__ TwF tw_factored(const TwF *shA, const TwF *shB, int line, int sp, long i, double q,
                                           double qi)
{
    const TwF a = shA[line * 8 + sp];
    const TwF b = shB[(1 << sp) - 1 + (int)(i & ((1l << sp) - 1))];
    TwF t;
    t.w = mulm_fp(a.w, b.w, b.c, q);
    t.c = t.w * qi;
    return t;
}

// PX: the first phase's words were loaded by the caller into px (position k of
// iteration it at px[(it << R) + k])
template <int LOGN, int PASS, bool FWD, int R, int LS, bool FIRST, bool LAST, bool PX, class IN, class OUT, class PB>
__device__ __forceinline__ void ntt_phase_fp(double *sh, const Blk &bk, long blk, const TwF *tw, const TwF *shA,
                                             const TwF *shB, const IN &in, const OUT &out, PB &pre, const double *px)
{
    typedef PhaseIdx<LOGN, PASS, R, LS> I;
    typedef NttGeo<LOGN> G;
    const double q = bk.pc->qd, qi = bk.pc->qinvd;
    if constexpr (LAST) prepare_pre(out, bk, pre);
#pragma unroll
    for (int it = 0; it < I::ITERS; it++) {
        I ix;
        if (!(OpaqueTid<OUT>::value ? ix.set(it, blk, bk.tid) : ix.set(it, blk))) break;
        double x[1 << R];
        if constexpr (FIRST && (std::is_same<IN, InBconv>::value || std::is_same<IN, InRescale>::value ||
                      std::is_same<IN, InBconvRs>::value)) {
            long g[1 << R];
#pragma unroll
            for (int k = 0; k < (1 << R); k++) g[k] = ix.gidx(k);
            in.template load_many_d<(1 << R)>(bk, g, x);
        } else {
#pragma unroll
            for (int k = 0; k < (1 << R); k++)
                x[k] = FIRST ? (PX ? px[(it << R) + k] : load_fp(in, bk, ix.gidx(k))) : sh[ix.lidx(k)];
        }
        if (FWD) {
#pragma unroll
            for (int h = R - 1; h >= 0; h--) {
                const long ib = ix.tw0(h);
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = ib + (k >> (h + 1));
                    const int sp = G::LC - 1 - LS - h;
                    const TwF t = PASS == 2 ? tw_factored(shA, shB, ix.line, sp, idx - (1l << (G::LR + sp)), q, qi)
                                            : tw[idx];
                    const double r = mulm_fp(x[k + (1 << h)], t.w, t.c, q);
                    const double a = x[k];
                    x[k] = a + r;
                    x[k + (1 << h)] = a - r;
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < R; h++) {
                const long ib = ix.tw0(h);
#pragma unroll
                for (int k = 0; k < (1 << R); k++) {
                    if (k & (1 << h)) continue;
                    const long idx = ib + (k >> (h + 1));
                    const int sp = G::LC - 1 - LS - h;
                    const TwF t = PASS == 2 ? tw_factored(shA, shB, ix.line, sp, idx - (1l << (G::LR + sp)), q, qi)
                                            : tw[idx];
                    const double a = x[k], b = x[k + (1 << h)];
                    const double sm = a + b;
                    x[k] = __fma_rn(-rint(sm * qi), q, sm);
                    x[k + (1 << h)] = mulm_fp(a - b, t.w, t.c, q);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < (1 << R); k++) {
            if (LAST) store_fp(out, bk, ix.gidx(k), x[k], pre.v[LAST ? (it << R) + k : 0]);
            else sh[ix.lidx(k)] = x[k];
        }
    }
}

// phase plan: radix-8 phases, forward 3,3,..,rem; inverse rem,..,3,3
// (radix-16 phases need up to 140 VGPRs in the fused variants and measured
// slower)
constexpr int RMAX = 3;
template <int LP, bool FWD, int PH>
struct PhasePlan {
    static constexpr int NPH = (LP + RMAX - 1) / RMAX;
    static constexpr int REM = LP - RMAX * (NPH - 1);
    static constexpr int R = FWD ? (PH < NPH - 1 ? RMAX : REM) : (PH == 0 ? REM : RMAX);
    static constexpr int BEFORE = FWD ? RMAX * PH : (PH == 0 ? 0 : REM + RMAX * (PH - 1));
    static constexpr int LS = FWD ? LP - BEFORE - R : BEFORE;
};

template <int LOGN, int PASS, bool FWD>
struct LastPhase {
    static constexpr int LP = PASS == 1 ? NttGeo<LOGN>::LR : NttGeo<LOGN>::LC;
    typedef PhasePlan<LP, FWD, PhasePlan<LP, FWD, 0>::NPH - 1> P;
    typedef PhaseIdx<LOGN, PASS, P::R, P::LS> I;
    static constexpr int NPOS = I::ITERS << P::R;
};

template <int LOGN, int PASS, bool FWD, int PH, class IN, class OUT, class PB>
__device__ __forceinline__ void ntt_phases(u64 *sh, const Blk &bk, long blk, const u64 *w, const u64 *wp,
                                           const IN &in, const OUT &out, PB &pre)
{
    typedef NttGeo<LOGN> G;
    constexpr int LP = PASS == 1 ? G::LR : G::LC;
    typedef PhasePlan<LP, FWD, PH> P;
    constexpr bool first = PH == 0, last = PH == P::NPH - 1;
    ntt_phase<LOGN, PASS, FWD, P::R, P::LS, first, last, IN, OUT>(sh, bk, blk, w, wp, in, out, pre);
    if constexpr (!last) {
        __syncthreads();
        ntt_phases<LOGN, PASS, FWD, PH + 1, IN, OUT>(sh, bk, blk, w, wp, in, out, pre);
    }
}

template <int LOGN, int PASS, bool FWD, int PH, bool PX, class IN, class OUT, class PB>
__device__ __forceinline__ void ntt_phases_fp(double *sh, const Blk &bk, long blk, const TwF *tw, const TwF *shA,
                                              const TwF *shB, const IN &in, const OUT &out, PB &pre,
                                              const double *px)
{
    typedef NttGeo<LOGN> G;
    constexpr int LP = PASS == 1 ? G::LR : G::LC;
    typedef PhasePlan<LP, FWD, PH> P;
    constexpr bool first = PH == 0, last = PH == P::NPH - 1;
    ntt_phase_fp<LOGN, PASS, FWD, P::R, P::LS, first, last, PX && first, IN, OUT>(sh, bk, blk, tw, shA, shB, in, out,
                                                                                  pre, px);
    if constexpr (!last) {
        __syncthreads();
        ntt_phases_fp<LOGN, PASS, FWD, PH + 1, false, IN, OUT>(sh, bk, blk, tw, shA, shB, in, out, pre, nullptr);
    }
}

// Whether k_ntt loads its row pass's first phase ahead of the factor tables
// and keeps a private copy of the prime's constants: not for the ModDown
// tail, which already holds three prefetched words per position (measured
// slower with the first phase loaded early, and the copy makes it spill)
template <class OUT>
struct RowPreload {
    static constexpr bool value = !std::is_same<OUT, OutModdownFin>::value;
};

// The words of a row pass's first phase (pass 2), loaded ahead of the block's
// LDS set-up so that their reads overlap the factor-table reads and barrier
template <int LOGN, bool FWD>
struct RowFirst {
    typedef PhasePlan<NttGeo<LOGN>::LC, FWD, 0> P;
    typedef PhaseIdx<LOGN, 2, P::R, P::LS> I;
    static constexpr int NX = I::ITERS << P::R;
    template <class IN>
    __device__ __forceinline__ static void load(const IN &in, const Blk &bk, long blk, int tid, double *px)
    {
#pragma unroll
        for (int it = 0; it < I::ITERS; it++) {
            I ix;
            if (!ix.set(it, blk, tid)) break;
#pragma unroll
            for (int k = 0; k < (1 << P::R); k++) px[(it << P::R) + k] = load_fp(in, bk, ix.gidx(k));
        }
    }
};

// minimum waves per SIMD the compiler must leave room for: the ModDown tail
// holds three prefetched words per position and would otherwise take just
// over 128 VGPRs (3 waves per SIMD instead of 4).  (Holding the conversion
// pass to 96 VGPRs for 5 waves spills and measured no faster than 4 waves.)
template <class IN, class OUT> struct NttWaves { static constexpr int value = 1; };
template <class IN> struct NttWaves<IN, OutModdownFin> { static constexpr int value = 4; };
// the conversion with the rescale term: one more word per position (else 132 VGPRs, 3 waves)
template <> struct NttWaves<InBconvRs, OutMid> { static constexpr int value = 4; };

// own_w > 0: polynomial p of the set is key-switch digit j = p mod own_ndig;
// its own limbs [j own_w, min(j own_w + own_w, own_nq)) are skipped
template <int LOGN, int PASS, bool FWD, class IN, class OUT>
__global__ void __launch_bounds__(256, (NttWaves<IN, OUT>::value)) k_ntt(NttTables T, PolySet ps, LimbMap lm, int skip_lo, int skip_hi,
                                             int own_w, int own_nq, int own_ndig, IN in, OUT out)
{
    typedef NttGeo<LOGN> G;
    constexpr int LT = PASS == 1 ? G::LR + G::LTC : G::LC + G::LRB;
    static_assert(PASS == 1 || G::LC == 8, "second-pass twiddle factors assume 256-word rows");
    // pass 2: the tile, then the twiddle factors B (256 pairs) and A (8 per row)
    constexpr int TWW = PASS == 2 ? 2 * (256 + 8 * (1 << G::LRB)) : 0;
    __shared__ u64 sh[(1 << LT) + TWW];
    // pass 1 runs the limbs of one polynomial back to back (limb fastest), so
    // blocks that read the same sources (basis conversion, rescale input) for
    // the same column tile share an XCD's L2; pass 2 runs the polynomials of
    // one limb back to back, sharing that prime's twiddle slice
    const int y = blockIdx.y;
    const int nll = gridDim.y / ps.npoly;
    const int poly = PASS == 1 ? y / nll : y % ps.npoly;
    const int li = PASS == 1 ? y % nll : y / ps.npoly;
    const int limb = li < skip_lo ? li : li + (skip_hi - skip_lo);
    if (own_w > 0) {
        const int j = poly % own_ndig;
        if (limb >= j * own_w && limb < min(j * own_w + own_w, own_nq)) return;
    }
    const int pi = lm.prime(limb);
    Blk bk;
    bk.a = ps.base + (long)limb * ps.lstride + (long)poly * ps.pstride;
    bk.limb = limb;
    bk.poly = poly;
    // a private copy of the prime's constants: held in registers, so the
    // phases' barriers (which order memory) do not make them be read again
    PrimeConst pcl;
    if constexpr (RowPreload<OUT>::value) {
        pcl = T.pc[pi];
        bk.pc = &pcl;
    } else {
        bk.pc = T.pc + pi;
    }
    bk.logN = LOGN;
    typedef LastPhase<LOGN, PASS, FWD> LPh;
    PreBuf<OUT::NPRE, LPh::NPOS> pre;
    if constexpr (OUT::NPRE > 0) {
#pragma unroll
        for (int it = 0; it < LPh::I::ITERS; it++) {
            typename LPh::I ix;
            if (!ix.set(it, (long)blockIdx.x)) break;
#pragma unroll
            for (int k = 0; k < (1 << LPh::P::R); k++) out.fetch(bk, ix.gidx(k), pre.v[(it << LPh::P::R) + k]);
        }
    }
    if (bk.pc->fp) {
        const TwF *tw = (FWD ? T.ffw : T.fiw) + ((long)pi << LOGN);
        TwF *shB = reinterpret_cast<TwF *>(sh + (1 << LT)), *shA = shB + 256;
        if constexpr (PASS == 2) {
            static_assert(!OpaqueTid<OUT>::value, "row pass of k_ntt indexes by threadIdx.x");
            constexpr bool early = RowPreload<OUT>::value;
            double px[RowFirst<LOGN, FWD>::NX];
            if constexpr (early) RowFirst<LOGN, FWD>::load(in, bk, (long)blockIdx.x, (int)threadIdx.x, px);
            // the prime's B table and the block's rows of A, read once into LDS
            const TwF *gB = (FWD ? T.fb : T.ib) + (long)pi * 256;
            const TwF *gA = (FWD ? T.fa : T.ia) + (((long)pi << G::LR) + ((long)blockIdx.x << G::LRB)) * 8;
            const int t = (int)threadIdx.x;
            if constexpr (early) {
                // both reads issued before either is used: the A index wraps, every
                // thread reads and stores an entry of the block's rows (threads
                // whose indices differ by a multiple of 8 2^LRB store the same
                // value at the same place)
                static_assert(8 * (1 << G::LRB) <= 256, "one A entry per thread at most");
                const int ta = t & (8 * (1 << G::LRB) - 1);
                const TwF vb = gB[t], va = gA[ta];
                shB[t] = vb;
                shA[ta] = va;
            } else {
                shB[t] = gB[t];
                if (t < 8 * (1 << G::LRB)) shA[t] = gA[t];
            }
            __syncthreads();
            ntt_phases_fp<LOGN, PASS, FWD, 0, early, IN, OUT>(reinterpret_cast<double *>(sh), bk, (long)blockIdx.x, tw,
                                                              shA, shB, in, out, pre, px);
        } else {
            ntt_phases_fp<LOGN, PASS, FWD, 0, false, IN, OUT>(reinterpret_cast<double *>(sh), bk, (long)blockIdx.x,
                                                              tw, shA, shB, in, out, pre, nullptr);
        }
        return;
    }
    const u64 *w = (FWD ? T.fw : T.iw) + ((long)pi << LOGN);
    const u64 *wp = (FWD ? T.fwp : T.iwp) + ((long)pi << LOGN);
    ntt_phases<LOGN, PASS, FWD, 0, IN, OUT>(sh, bk, (long)blockIdx.x, w, wp, in, out, pre);
}

// ModUp's second pass fused with the key inner product, for the limbs on FP64
// primes: a block owns one (limb, row tile) of one batch element and runs the
// forward row pass of every digit's extended polynomial in turn (the digit's
// own limb is the input polynomial itself, already in NTT form); each result
// is left in LDS and multiplied there by the digit's two key words (standard
// form, doubles), the products summed in registers, so the extended digits
// never reach HBM; the two sums are stored reduced to [0, q).  A thread owns
// tile words threadIdx.x + 256 k, so key, input and output accesses are
// coalesced.  c = w / q is formed as w fl(1/q): each product is then within
// q + 2^37 of zero and 16 digits stay below 2^50.  Blocks are taken in spans
// of gspan (limb, tile) groups, element by element: block ((s nb + e) gspan +
// r) runs group s gspan + r of element e.  With gspan a multiple of 8 the
// blocks of one group and different elements land on one XCD (hardware block
// b runs on XCD b mod 8), so the tile's key words come from HBM once and then
// from L2; gspan = 1 puts the elements of a group side by side instead.
// mid: pass-1 output, limb t of polynomial p (= e ndig + j) at mid + t mid_ls + p mid_ps;
// d: limb t of element e at d + t d_ls + e d_es; kf: digit j, component c, limb t at
// kf + j kf_ds + c kf_cs + t N (doubles); acc: element e component c limb t at
// acc + e acc_es + c acc_cs + t N.
template <int LOGN>
__global__ void __launch_bounds__(256, 4) k_modup_keyip(NttTables T, const u64 *mid, long mid_ls, long mid_ps,
                                                        const u64 *d, long d_ls, long d_es, const double *kf,
                                                        long kf_ds, long kf_cs, u64 *acc, long acc_es, long acc_cs,
                                                        int ndig, int w, int nb, int limb_lo, int ngroups,
                                                        int gspan)
{
    typedef NttGeo<LOGN> G;
    static_assert(G::LC == 8, "row tiles of 256-word rows");
    constexpr int LT = G::LC + G::LRB;
    constexpr int TWW = 2 * (256 + 8 * (1 << G::LRB));
    constexpr long N = 1l << LOGN;
    constexpr int TILES = 1 << (G::LR - G::LRB);
    constexpr int NP = (1 << LT) / 256;  // words per thread
    __shared__ u64 sh[(1 << LT) + TWW];
    double *shd = reinterpret_cast<double *>(sh);
    const int b = (int)blockIdx.x, i = b / gspan;
    const int e = i % nb, grp = (i / nb) * gspan + b % gspan;
    if (grp >= ngroups) return;
    const int limb = limb_lo + grp / TILES;
    const long tile = grp % TILES;
    Blk bk;
    bk.limb = limb;
    const PrimeConst pcl = T.pc[limb];  // Q limbs: limb index = prime index; kept in registers
    bk.pc = &pcl;
    bk.logN = LOGN;
    const double q = bk.pc->qd, qi = bk.pc->qinvd;
    const TwF *tw = T.ffw + ((long)limb << LOGN);
    TwF *shB = reinterpret_cast<TwF *>(sh + (1 << LT)), *shA = shB + 256;
    bool tables = false;
    double a0[NP], a1[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) a0[k] = a1[k] = 0.0;
    const int jown = limb / w;
    for (int j = 0; j < ndig; j++) {
        const double *k0 = kf + j * kf_ds + (long)limb * N, *k1 = k0 + kf_cs;
        // a fresh copy of the thread index per digit: the transform's addresses
        // are recomputed per digit instead of all being kept live across the loop
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        const long g0 = (tile << LT) + tid;
        if (j == jown) {
            const u64 *dp = d + (long)limb * d_ls + (long)e * d_es;
#pragma unroll
            for (int k = 0; k < NP; k++) {
                const long g = g0 + 256 * k;
                const double x = u2d(dp[g]), w0 = k0[g], w1 = k1[g];
                a0[k] += mulm_fp(x, w0, w0 * qi, q);
                a1[k] += mulm_fp(x, w1, w1 * qi, q);
            }
            continue;
        }
        bk.poly = e * ndig + j;
        bk.a = const_cast<u64 *>(mid) + (long)limb * mid_ls + (long)bk.poly * mid_ps;
        bk.tid = tid;
        // the digit's first-phase words are requested before the barrier (and,
        // for the first digit, before the factor tables), so their reads overlap
        double px[RowFirst<LOGN, true>::NX];
        RowFirst<LOGN, true>::load(InMid(), bk, tile, tid, px);
        if (!tables) {
            const TwF *gB = T.fb + (long)limb * 256;
            const TwF *gA = T.fa + (((long)limb << G::LR) + (tile << G::LRB)) * 8;
            const int t = (int)threadIdx.x;
            // both reads issued before either is used: the A index wraps, every
            // thread reads and stores an entry of the block's rows (threads whose
            // indices differ by a multiple of 8 2^LRB store the same value at the
            // same place)
            static_assert(8 * (1 << G::LRB) <= 256, "one A entry per thread at most");
            const int ta = t & (8 * (1 << G::LRB) - 1);
            const TwF vb = gB[t], va = gA[ta];
            shB[t] = vb;
            shA[ta] = va;
            tables = true;
        }
        __syncthreads();  // factor tables in place; the previous digit's LDS reads are done
        PreBuf<0, 1> none;
        ntt_phases_fp<LOGN, 2, true, 0, true, InMid, OutLds>(shd, bk, tile, tw, shA, shB, InMid(),
                                                              OutLds{shd, (1 << LT) - 1}, none, px);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const long g = g0 + 256 * k;
            const double x = shd[OutLds::word(tid + 256 * k)], w0 = k0[g], w1 = k1[g];
            a0[k] += mulm_fp(x, w0, w0 * qi, q);
            a1[k] += mulm_fp(x, w1, w1 * qi, q);
        }
    }
    u64 *o0 = acc + (long)e * acc_es + (long)limb * N, *o1 = o0 + acc_cs;
    const long g0 = (tile << LT) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const long g = g0 + 256 * k;
        o0[g] = d2u_mod(a0[k], q, qi);
        o1[g] = d2u_mod(a1[k], q, qi);
    }
}

// ---------------------------------------------------------------- launchers
struct NttJob {
    PolySet ps;
    LimbMap lm;
    int skip_lo = 0, skip_hi = 0, own_w = 0, own_nq = 0, own_ndig = 1;
};

template <int LOGN, class IN, class OUT>
static void fwd_n(const NttTables &t, const NttJob &j, const IN &in, const OUT &out, hipStream_t s, KernelTimer *tm)
{
    typedef NttGeo<LOGN> G;
    const int nl = j.ps.nl - (j.skip_hi - j.skip_lo);
    dim3 blk(256), g1(1 << (G::LC - G::LTC), nl * j.ps.npoly), g2(1 << (G::LR - G::LRB), nl * j.ps.npoly);
    // limb-polynomials transformed (a key-switch digit's own limbs are skipped)
    const double polys = (double)nl * j.ps.npoly - (j.own_w > 0 ? (double)(j.ps.npoly / j.own_ndig) * j.own_nq : 0.0);
    const double wb = 8.0 * (double)(1l << LOGN);
    const double bytes1 = wb * (in.read_words(j.ps.npoly, nl) + polys);
    const double bytes2 = wb * (2.0 * polys + out.extra_words(j.ps.npoly, nl));
    if constexpr (G::LR > 0) {
        bool on = tm && tm->on(KID_NTT_FWD1);
        if (on) tm->before(s);
        hipLaunchKernelGGL((k_ntt<LOGN, 1, true, IN, OutMid>), g1, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, in, OutMid());
        if (on) tm->after(s, bytes1, polys * (double)(1l << (LOGN - 1)) * G::LR);
        on = tm && tm->on(KID_NTT_FWD2);
        if (on) tm->before(s);
        hipLaunchKernelGGL((k_ntt<LOGN, 2, true, InMid, OUT>), g2, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, InMid(), out);
        if (on) tm->after(s, bytes2, polys * (double)(1l << (LOGN - 1)) * G::LC);
    } else {
        (void)g1;
        (void)bytes1;
        (void)bytes2;
        hipLaunchKernelGGL((k_ntt<LOGN, 2, true, IN, OUT>), g2, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, in, out);
    }
}

template <int LOGN, class IN, class OUT>
static void inv_n(const NttTables &t, const NttJob &j, const IN &in, const OUT &out, hipStream_t s, KernelTimer *tm)
{
    typedef NttGeo<LOGN> G;
    const int nl = j.ps.nl - (j.skip_hi - j.skip_lo);
    dim3 blk(256), g1(1 << (G::LC - G::LTC), nl * j.ps.npoly), g2(1 << (G::LR - G::LRB), nl * j.ps.npoly);
    const double polys = (double)nl * j.ps.npoly, wb = 8.0 * (double)(1l << LOGN);
    const double bytes2 = wb * (in.read_words(j.ps.npoly, nl) + polys);
    const double bytes1 = wb * (2.0 * polys + out.extra_words(j.ps.npoly, nl));
    if constexpr (G::LR > 0) {
        bool on = tm && tm->on(KID_NTT_INV2);
        if (on) tm->before(s);
        hipLaunchKernelGGL((k_ntt<LOGN, 2, false, IN, OutMid>), g2, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, in, OutMid());
        if (on) tm->after(s, bytes2, polys * (double)(1l << (LOGN - 1)) * G::LC);
        on = tm && tm->on(KID_NTT_INV1);
        if (on) tm->before(s);
        hipLaunchKernelGGL((k_ntt<LOGN, 1, false, InMid, OUT>), g1, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, InMid(), out);
        if (on) tm->after(s, bytes1, polys * (double)(1l << (LOGN - 1)) * G::LR);
    } else {
        (void)g1;
        (void)bytes1;
        (void)bytes2;
        hipLaunchKernelGGL((k_ntt<LOGN, 2, false, IN, OUT>), g2, blk, 0, s, t, j.ps, j.lm, j.skip_lo, j.skip_hi,
                           j.own_w, j.own_nq, j.own_ndig, in, out);
    }
}

#define NTT_DISPATCH(FN, ...)                                                                  \
    switch (t.logN) {                                                                          \
    case 10: FN<10>(__VA_ARGS__); break;                                                       \
    case 11: FN<11>(__VA_ARGS__); break;                                                       \
    case 12: FN<12>(__VA_ARGS__); break;                                                       \
    case 13: FN<13>(__VA_ARGS__); break;                                                       \
    case 14: FN<14>(__VA_ARGS__); break;                                                       \
    case 15: FN<15>(__VA_ARGS__); break;                                                       \
    case 16: FN<16>(__VA_ARGS__); break;                                                       \
    default: break;                                                                            \
    }

template <int LOGN>
static void plain_n(const NttTables &t, const NttJob &j, bool inverse, hipStream_t s, KernelTimer *tm)
{
    if (!inverse) fwd_n<LOGN>(t, j, InWork(), OutWork<OW_REDUCE>(), s, tm);
    else inv_n<LOGN>(t, j, InWork(), OutWork<OW_SCALE_N>(), s, tm);
}

void launch_ntt(const NttTables &t, PolySet ps, LimbMap lm, int skip_lo, int skip_hi, bool inverse,
                hipStream_t s, KernelTimer *tm)
{
    NttJob j;
    j.ps = ps;
    j.lm = lm;
    j.skip_lo = skip_lo;
    j.skip_hi = skip_hi;
    if (ps.nl - (skip_hi - skip_lo) <= 0) return;
    NTT_DISPATCH(plain_n, t, j, inverse, s, tm);
}

// inverse transform of `src` (read through sigma_galois if galois > 1) into the
// working set ps, every limb multiplied by scale[limb] (N^-1 folded in)
template <int LOGN>
static void intt_src_n(const NttTables &t, const NttJob &j, const InSrc &in, const OutScaleTab &o, hipStream_t s,
                       KernelTimer *tm)
{
    if (o.s) inv_n<LOGN>(t, j, in, o, s, tm);
    else inv_n<LOGN>(t, j, in, OutWork<OW_SCALE_N>(), s, tm);
}

void launch_intt_from(const NttTables &t, PolySet work, LimbMap lm, const u64 *src, long src_ls, long src_ps,
                      u64 galois, const u64 *scale, const u64 *scalep, hipStream_t s, KernelTimer *tm)
{
    NttJob j;
    j.ps = work;
    j.lm = lm;
    InSrc in{src, src_ls, src_ps, galois};
    OutScaleTab o{scale, scalep};
    NTT_DISPATCH(intt_src_n, t, j, in, o, s, tm);
}

template <int LOGN>
static void intt_modup_n(const NttTables &t, const NttJob &j, const InSrc &in, const OutScaleTabFp &o,
                         hipStream_t s, KernelTimer *tm)
{
    inv_n<LOGN>(t, j, in, o, s, tm);
}

void launch_intt_modup(const NttTables &t, PolySet work, LimbMap lm, const u64 *src, long src_ls, long src_ps,
                       const u64 *scale, const u64 *scalep, const TwF *scalef, hipStream_t s, KernelTimer *tm)
{
    NttJob j;
    j.ps = work;
    j.lm = lm;
    InSrc in{src, src_ls, src_ps, 0};
    OutScaleTabFp o{scale, scalep, scalef};
    NTT_DISPATCH(intt_modup_n, t, j, in, o, s, tm);
}

// ModUp of all digits: ext is [ndig][next][N]; the forward transform of every
// non-own limb of every digit starts from the fast basis conversion of the
// digit's inverse-hat-scaled coefficients y (limb stride N)
template <int LOGN>
static void modup_n(const NttTables &t, const NttJob &j, const InBconv &in, hipStream_t s, KernelTimer *tm)
{
    fwd_n<LOGN>(t, j, in, OutWork<OW_REDUCE>(), s, tm);
}

void launch_modup(const NttTables &t, u64 *ext, int ndig, int nq, int alpha, int w, int nb, LimbMap lm,
                  const u64 *y, const u64 *hatm, const TwF *hatf, const u64 wide[2], const u64 dbl[2],
                  hipStream_t s, KernelTimer *tm)
{
    const long N = 1l << t.logN;
    const int next = nq + alpha;
    NttJob j;
    j.ps = PolySet{ext, N, (long)next * N, next, ndig * nb};
    j.lm = lm;
    j.own_w = w;
    j.own_nq = nq;
    j.own_ndig = ndig;
    InBconv in;
    in.src = y;
    in.src_bs = (long)nq * N;
    in.src_ps = (long)w * N;
    in.ndig = ndig;
    in.hatm = hatm;
    in.hat_ps = (long)w * next;
    in.hat_ks = next;
    in.ns_fixed = 0;
    in.w = w;
    in.nq = nq;
    in.hatf = hatf;
    in.wide[0] = wide[0];
    in.wide[1] = wide[1];
    in.dbl[0] = dbl[0];
    in.dbl[1] = dbl[1];
    NTT_DISPATCH(modup_n, t, j, in, s, tm);
}

// ModUp with the key inner product fused into its second pass on the FP64
// limbs [fp_lo, fp_hi): pass 1 for every non-own limb, pass 2 (stored) on the
// other limbs, then k_modup_keyip on the FP64 limbs
template <int LOGN>
static void modup_keyip_n(const NttTables &t, const NttJob &j, const InBconv &in, const ModupKeyipArgs &a,
                          hipStream_t s, KernelTimer *tm)
{
    typedef NttGeo<LOGN> G;
    static_assert(G::LR > 0, "two passes");
    const int nl = j.ps.nl, np = j.ps.npoly;
    const double wb = 8.0 * (double)(1l << LOGN);
    const double own = (double)(np / j.own_ndig) * j.own_nq;
    dim3 blk(256), g1(1 << (G::LC - G::LTC), nl * np);
    bool on = tm && tm->on(KID_NTT_FWD1);
    if (on) tm->before(s);
    hipLaunchKernelGGL((k_ntt<LOGN, 1, true, InBconv, OutMid>), g1, blk, 0, s, t, j.ps, j.lm, 0, 0, j.own_w, j.own_nq,
                       j.own_ndig, in, OutMid());
    if (on) tm->after(s, wb * (in.read_words(np, nl) + (double)nl * np - own),
                      ((double)nl * np - own) * (double)(1l << (LOGN - 1)) * G::LR);
    const int nfp = a.fp_hi - a.fp_lo, nli = nl - nfp;
    // integer-prime limbs: the second pass stores the extended digits (own limbs skipped: 1 per
    // element for the one own limb outside [fp_lo, fp_hi), the base prime)
    dim3 g2(1 << (G::LR - G::LRB), nli * np);
    on = tm && tm->on(KID_NTT_FWD2);
    if (on) tm->before(s);
    hipLaunchKernelGGL((k_ntt<LOGN, 2, true, InMid, OutWork<OW_REDUCE>>), g2, blk, 0, s, t, j.ps, j.lm, a.fp_lo,
                       a.fp_hi, j.own_w, j.own_nq, j.own_ndig, InMid(), OutWork<OW_REDUCE>());
    const double pi2 = (double)nli * np - (double)(np / j.own_ndig) * a.own_int;
    if (on) tm->after(s, wb * 2.0 * pi2, pi2 * (double)(1l << (LOGN - 1)) * G::LC);
    constexpr int TILES = 1 << (G::LR - G::LRB);
    const int ngroups = nfp * TILES;
    on = tm && tm->on(KID_MODUP_KEYIP);
    if (on) tm->before(s);
    const int gs = a.gspan > 0 ? a.gspan : 8;
    hipLaunchKernelGGL((k_modup_keyip<LOGN>), dim3(((ngroups + gs - 1) / gs) * gs * a.nb), blk, 0, s, t, j.ps.base,
                       j.ps.lstride, j.ps.pstride, a.d, a.d_ls, a.d_es, a.kf, a.kf_ds, a.kf_cs, a.acc, a.acc_es,
                       a.acc_cs, j.own_ndig, j.own_w, a.nb, a.fp_lo, ngroups, gs);
    // per limb and element: ndig words read (pass-1 output or the input limb), two written;
    // per limb: 2 ndig key words
    if (on) tm->after(s, wb * nfp * ((double)a.nb * j.own_ndig + 2.0 * j.own_ndig + 2.0 * a.nb),
                      (double)nfp * a.nb * (double)(1l << (LOGN - 1)) * G::LC * (j.own_ndig - 1));
}

void launch_modup_keyip(const NttTables &t, u64 *ext, int ndig, int nq, int alpha, int w, int nb, LimbMap lm,
                        const u64 *y, const u64 *hatm, const TwF *hatf, const u64 wide[2], const u64 dbl[2],
                        const ModupKeyipArgs &a, hipStream_t s, KernelTimer *tm)
{
    const long N = 1l << t.logN;
    const int next = nq + alpha;
    NttJob j;
    j.ps = PolySet{ext, N, (long)next * N, next, ndig * nb};
    j.lm = lm;
    j.own_w = w;
    j.own_nq = nq;
    j.own_ndig = ndig;
    InBconv in;
    in.src = y;
    in.src_bs = (long)nq * N;
    in.src_ps = (long)w * N;
    in.ndig = ndig;
    in.hatm = hatm;
    in.hat_ps = (long)w * next;
    in.hat_ks = next;
    in.ns_fixed = 0;
    in.w = w;
    in.nq = nq;
    in.hatf = hatf;
    in.wide[0] = wide[0];
    in.wide[1] = wide[1];
    in.dbl[0] = dbl[0];
    in.dbl[1] = dbl[1];
    NTT_DISPATCH(modup_keyip_n, t, j, in, a, s, tm);
}

// ModDown: yP [2][alpha][N] (inverse-hat-scaled P limbs, coefficient form) ->
// forward transform of the conversion to Q_l, tail fused into the last store
template <int LOGN>
static void moddown_n(const NttTables &t, const NttJob &j, const InBconv &in, const OutModdownFin &o, hipStream_t s,
                      KernelTimer *tm)
{
    fwd_n<LOGN>(t, j, in, o, s, tm);
}

void launch_moddown(const NttTables &t, u64 *tmp, int nq, int alpha, int npoly, LimbMap lm, const u64 *yP,
                    const u64 *hatm, long hat_ks, const OutModdownArgs &a, hipStream_t s, KernelTimer *tm)
{
    const long N = 1l << t.logN;
    NttJob j;
    j.ps = PolySet{tmp, N, (long)nq * N, nq, npoly};
    j.lm = lm;
    InBconv in;
    in.src = yP;
    in.src_bs = (long)alpha * N;
    in.src_ps = 0;
    in.ndig = 1;
    in.hatm = hatm;
    in.hat_ps = 0;
    in.hat_ks = hat_ks;
    in.ns_fixed = alpha;
    in.w = 0;
    in.nq = nq;
    // every source is a special prime: the integer conversion is as cheap here
    in.hatf = nullptr;
    in.wide[0] = in.wide[1] = 0;
    in.dbl[0] = in.dbl[1] = 0;
    OutModdownFin o{a.acc, a.acc_ls, a.acc_ps, a.base, a.bls, a.bes, a.bcs, a.mask, a.galois, a.out, a.ols, a.ops,
                    a.pinv, a.pinvp, a.add, a.als, a.aes, a.pinvf};
    NTT_DISPATCH(moddown_n, t, j, in, o, s, tm);
}

template <int LOGN>
static void moddown_rescale_n(const NttTables &t, const NttJob &j, const InBconvRs &in,
                              const OutModdownRescaleFin &o, hipStream_t s, KernelTimer *tm)
{
    fwd_n<LOGN>(t, j, in, o, s, tm);
}

void launch_moddown_rescale(const NttTables &t, u64 *tmp, int l, int alpha, int npoly, const u64 *yP,
                            const u64 *hatm, long hat_ks, const u64 *last, u64 ql, const u64 *pm, const u64 *pmp,
                            const TwF *pmf, const OutModdownRescaleArgs &a, int L1, hipStream_t s, KernelTimer *tm)
{
    const long N = 1l << t.logN;
    NttJob j;
    j.ps = PolySet{tmp, N, (long)l * N, l, npoly};
    j.lm = LimbMap{l, L1, 0};
    InBconvRs in;
    in.src = yP;
    in.src_bs = (long)alpha * N;
    in.src_ps = 0;
    in.ndig = 1;
    in.hatm = hatm;
    in.hat_ps = 0;
    in.hat_ks = hat_ks;
    in.ns_fixed = alpha;
    in.w = 0;
    in.nq = l;
    in.hatf = nullptr;
    in.wide[0] = in.wide[1] = 0;
    in.dbl[0] = in.dbl[1] = 0;
    in.last = last;
    in.last_ps = N;
    in.ql = ql;
    const bool small = ql < (1ull << 52);
    in.qld = small ? (double)ql : 0.0;
    in.hd = small ? (double)(ql >> 1) : 0.0;
    in.pm = pm;
    in.pmp = pmp;
    in.pmf = pmf;
    OutModdownRescaleFin o{a.acc, a.acc_ls, a.acc_ps, a.base, a.bls, a.bes, a.bcs, a.out, a.ols, a.ops,
                           a.pinv, a.pinvp, a.pinvf, a.inv, a.invp, a.invf, a.cadd};
    NTT_DISPATCH(moddown_rescale_n, t, j, in, o, s, tm);
}

// rescale of both polynomials: tmp [2][l][N] working set; last = dropped limb
// in coefficient form ([2][N]); out = (in - NTT(...)) q_l^-1
template <int LOGN>
static void rescale_n(const NttTables &t, const NttJob &j, const InRescale &in, const OutRescaleFin &o,
                      hipStream_t s, KernelTimer *tm)
{
    fwd_n<LOGN>(t, j, in, o, s, tm);
}

void launch_rescale_ntt(const NttTables &t, u64 *tmp, int l, int npoly, const u64 *last, u64 ql, const u64 *in,
                        long in_ls, long in_ps, u64 *out, long out_ls, long out_ps, const u64 *inv, const u64 *invp,
                        const TwF *invf, const u64 *pm, const u64 *pmp, const u64 *cadd, int L1, hipStream_t s,
                        KernelTimer *tm)
{
    const long N = 1l << t.logN;
    NttJob j;
    j.ps = PolySet{tmp, N, (long)l * N, l, npoly};
    j.lm = LimbMap{l, L1, 0};
    const bool small = ql < (1ull << 52);
    InRescale ir{last, N, ql, small ? (double)ql : 0.0, small ? (double)(ql >> 1) : 0.0};
    OutRescaleFin o{in, in_ls, in_ps, out, out_ls, out_ps, inv, invp, invf, pm, pmp, cadd};
    NTT_DISPATCH(rescale_n, t, j, ir, o, s, tm);
}

}  // namespace hk
