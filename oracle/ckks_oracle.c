/*
 * Plain CPU reference ("oracle") for the RNS-CKKS ring arithmetic that carries
 * the encrypted KAN inference of "Efficient Privacy-Preserving KAN Inference
 * Using Homomorphic Encryption" (Preliminaries, "Homomorphic Encryption":
 * ciphertext addition, multiplication and rotation under RNS-CKKS).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product never
 * does.  It shares no code with the GPU path.
 *
 * The paper names RNS-CKKS (Cheon, Han, Kim, Kim, Song, SAC 2018) but does not
 * describe its internals.  Everything below follows the textbook definitions:
 *   - polynomials in Z_q[X]/(X^N+1), kept in COEFFICIENT form, one array of N
 *     residues per RNS limb;
 *   - every modular product is a 128-bit product followed by the hardware
 *     remainder (slow and obviously correct);
 *   - negacyclic products go through a psi-twisted cyclic NTT;
 *   - fast basis conversion without overflow correction (full-RNS CKKS);
 *   - hybrid key switching with digits of `w` consecutive Q limbs and special
 *     modulus P (Han and Ki, CT-RSA 2020);
 *   - rescale by the last prime with rounding;
 *   - canonical-embedding encoding in double-double precision, rounded to the
 *     nearest integer with ties to even;
 *   - sampling from the ChaCha20 block function (RFC 8439).
 * Loops over independent RNS limbs (and, in the basis conversion, over
 * independent coefficients) may run on several host threads (OpenMP); each
 * iteration computes exactly what it computes alone, so the results do not
 * depend on the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;
typedef __int128 i128;

/* host threads used by the limb loops (0 or less: the OpenMP default) */
void oc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
int oc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* scalar modular arithmetic                                                   */
/* ------------------------------------------------------------------------- */
static u64 addm(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

u64 oc_powm(u64 a, u64 e, u64 q)
{
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulm(r, a, q);
        a = mulm(a, a, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime (Fermat) */
u64 oc_invm(u64 a, u64 q) { return oc_powm(a % q, q - 2, q); }

/* deterministic Miller-Rabin for 64-bit integers */
int oc_is_prime(u64 n)
{
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = oc_powm(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int r = 1; r < s; r++) {
            x = mulm(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* parameter generation                                                         */
/* ------------------------------------------------------------------------- */
static int in_list(u64 c, const u64 *l, int n)
{
    for (int i = 0; i < n; i++)
        if (l[i] == c) return 1;
    return 0;
}

/* the prime = 1 (mod M) nearest to T that is not in `used` (ties: the smaller) */
static u64 nearest_prime(double T, u64 M, const u64 *used, int nused)
{
    u64 klo = (u64)floor((T - 1.0) / (double)M);
    u64 khi = klo + 1;
    for (;;) {
        double dlo = T - (double)(klo * M + 1);
        double dhi = (double)(khi * M + 1) - T;
        if (dlo <= dhi) {
            u64 c = klo * M + 1;
            if (oc_is_prime(c) && !in_list(c, used, nused)) return c;
            klo--;
        } else {
            u64 c = khi * M + 1;
            if (oc_is_prime(c) && !in_list(c, used, nused)) return c;
            khi++;
        }
    }
}

/*
 * Prime chain for N = 2^logN.  All primes are 1 mod 2N (negacyclic NTT).
 *   q[0]      : largest prime below 2^base_bits;
 *   p[0..a-1] : the next largest primes below 2^special_bits (distinct);
 *   q[L..1]   : chosen top-down so that every level keeps a canonical scale
 *               close to Delta_l = 2^bits_l:  S_L = Delta_L,
 *               q_l = prime nearest (S_l*S_l)/Delta_l,  S_{l-1} = (S_l*S_l)/q_l,
 *               where bits_l = boot_bits for the top n_boot levels (l > L - n_boot,
 *               the levels a bootstrapping consumes) and scale_bits below;
 *               the top computation level takes S_{L-n_boot} = 2^scale_bits.
 * Writes S[0..L] (canonical scale of each level).  Returns 0.
 */
int oc_gen_primes(int logN, int base_bits, int n_scale, int scale_bits, int n_special,
                  int special_bits, int n_boot, int boot_bits, u64 *q, u64 *p, double *S)
{
    u64 M = 2ULL << logN;
    u64 used[256];
    int nused = 0;
    u64 k = ((1ULL << base_bits) - 2) / M;
    while (!oc_is_prime(k * M + 1)) k--;
    q[0] = k * M + 1;
    used[nused++] = q[0];
    u64 ks = ((1ULL << special_bits) - 2) / M;
    for (int i = 0; i < n_special; i++) {
        while (!oc_is_prime(ks * M + 1) || in_list(ks * M + 1, used, nused)) ks--;
        p[i] = ks * M + 1;
        used[nused++] = p[i];
        ks--;
    }
    int top_c = n_scale - n_boot; /* top computation level */
    double s = ldexp(1.0, n_boot > 0 ? boot_bits : scale_bits);
    S[n_scale] = s;
    for (int l = n_scale; l >= 1; l--) {
        double delta = ldexp(1.0, l > top_c ? boot_bits : scale_bits);
        double T = (s * s) / delta;
        q[l] = nearest_prime(T, M, used, nused);
        used[nused++] = q[l];
        s = (n_boot > 0 && l == top_c + 1) ? ldexp(1.0, scale_bits) : (s * s) / (double)q[l];
        S[l - 1] = s;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* negacyclic NTT tables (cached per (q, logN))                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    u64 q;
    int logN;
    u64 *psi;   /* psi^j, j < N            */
    u64 *ipsi;  /* psi^-j * N^-1, j < N    */
    u64 *w;     /* omega^j, j < N/2 (omega = psi^2) */
    u64 *iw;    /* omega^-j                 */
} ntt_tab;

#define MAX_TABS 256
static ntt_tab g_tabs[MAX_TABS];
static int g_ntabs = 0;

/* smallest psi of the form c^((q-1)/2N), c = 2,3,..., with psi^N = -1 */
u64 oc_find_psi(u64 q, int logN)
{
    u64 N = 1ULL << logN;
    for (u64 c = 2;; c++) {
        u64 psi = oc_powm(c, (q - 1) / (2 * N), q);
        if (oc_powm(psi, N, q) == q - 1) return psi;
    }
}

static const ntt_tab *make_tab(u64 q, int logN);
static const ntt_tab *get_tab(u64 q, int logN)
{
    const ntt_tab *r;
#pragma omp critical(oc_tabs)
    r = make_tab(q, logN);
    return r;
}

static const ntt_tab *make_tab(u64 q, int logN)
{
    for (int i = 0; i < g_ntabs; i++)
        if (g_tabs[i].q == q && g_tabs[i].logN == logN) return &g_tabs[i];
    if (g_ntabs == MAX_TABS) abort();
    ntt_tab *t = &g_tabs[g_ntabs];
    u64 N = 1ULL << logN;
    u64 psi = oc_find_psi(q, logN);
    u64 ipsi = oc_invm(psi, q);
    u64 ninv = oc_invm(N, q);
    t->q = q;
    t->logN = logN;
    t->psi = malloc(N * sizeof(u64));
    t->ipsi = malloc(N * sizeof(u64));
    t->w = malloc(N / 2 * sizeof(u64));
    t->iw = malloc(N / 2 * sizeof(u64));
    u64 a = 1, b = ninv;
    for (u64 j = 0; j < N; j++) {
        t->psi[j] = a;
        t->ipsi[j] = b;
        a = mulm(a, psi, q);
        b = mulm(b, ipsi, q);
    }
    u64 om = mulm(psi, psi, q), iom = oc_invm(om, q);
    a = 1;
    b = 1;
    for (u64 j = 0; j < N / 2; j++) {
        t->w[j] = a;
        t->iw[j] = b;
        a = mulm(a, om, q);
        b = mulm(b, iom, q);
    }
    g_ntabs++;
    return t;
}

/* textbook iterative radix-2 cyclic DFT over Z_q: A_k = sum_j a_j W^{jk} */
static void cyclic_ntt(u64 *a, int logN, u64 q, const u64 *wp)
{
    u64 N = 1ULL << logN;
    for (u64 i = 1, j = 0; i < N; i++) {
        u64 bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (u64 len = 2; len <= N; len <<= 1) {
        u64 half = len >> 1, step = N / len;
        for (u64 i = 0; i < N; i += len)
            for (u64 j = 0; j < half; j++) {
                u64 u = a[i + j], v = mulm(a[i + j + half], wp[j * step], q);
                a[i + j] = addm(u, v, q);
                a[i + j + half] = subm(u, v, q);
            }
    }
}

/* forward negacyclic transform: evaluations a(psi * omega^k) for k < N */
void oc_ntt_fwd(u64 *a, int logN, u64 q)
{
    const ntt_tab *t = get_tab(q, logN);
    u64 N = 1ULL << logN;
    for (u64 j = 0; j < N; j++) a[j] = mulm(a[j], t->psi[j], q);
    cyclic_ntt(a, logN, q, t->w);
}

/* inverse of oc_ntt_fwd */
void oc_ntt_inv(u64 *a, int logN, u64 q)
{
    const ntt_tab *t = get_tab(q, logN);
    u64 N = 1ULL << logN;
    cyclic_ntt(a, logN, q, t->iw);
    for (u64 j = 0; j < N; j++) a[j] = mulm(a[j], t->ipsi[j], q);
}

/* out = a * b in Z_q[X]/(X^N+1); out may alias a or b */
void oc_negacyclic_mul(const u64 *a, const u64 *b, u64 *out, int logN, u64 q)
{
    u64 N = 1ULL << logN;
    u64 *fa = malloc(N * sizeof(u64)), *fb = malloc(N * sizeof(u64));
    memcpy(fa, a, N * sizeof(u64));
    memcpy(fb, b, N * sizeof(u64));
    oc_ntt_fwd(fa, logN, q);
    oc_ntt_fwd(fb, logN, q);
    for (u64 j = 0; j < N; j++) fa[j] = mulm(fa[j], fb[j], q);
    oc_ntt_inv(fa, logN, q);
    memcpy(out, fa, N * sizeof(u64));
    free(fa);
    free(fb);
}

/* O(N^2) schoolbook negacyclic product, the definition the NTT must match */
void oc_schoolbook_mul(const u64 *a, const u64 *b, u64 *out, int logN, u64 q)
{
    u64 N = 1ULL << logN;
    u64 *acc = calloc(N, sizeof(u64));
    for (u64 i = 0; i < N; i++)
        for (u64 j = 0; j < N; j++) {
            u64 p = mulm(a[i], b[j], q);
            u64 k = i + j;
            if (k < N) acc[k] = addm(acc[k], p, q);
            else acc[k - N] = subm(acc[k - N], p, q);
        }
    memcpy(out, acc, N * sizeof(u64));
    free(acc);
}

/* ------------------------------------------------------------------------- */
/* RNS polynomial operations (arrays of nl limbs x N coefficients)              */
/* ------------------------------------------------------------------------- */
void oc_poly_add(const u64 *a, const u64 *b, u64 *out, int nl, int logN, const u64 *m)
{
    u64 N = 1ULL << logN;
    for (int i = 0; i < nl; i++)
        for (u64 j = 0; j < N; j++) out[i * N + j] = addm(a[i * N + j], b[i * N + j], m[i]);
}

void oc_poly_sub(const u64 *a, const u64 *b, u64 *out, int nl, int logN, const u64 *m)
{
    u64 N = 1ULL << logN;
    for (int i = 0; i < nl; i++)
        for (u64 j = 0; j < N; j++) out[i * N + j] = subm(a[i * N + j], b[i * N + j], m[i]);
}

void oc_poly_mul(const u64 *a, const u64 *b, u64 *out, int nl, int logN, const u64 *m)
{
    u64 N = 1ULL << logN;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nl; i++) oc_negacyclic_mul(a + i * N, b + i * N, out + i * N, logN, m[i]);
}

/* multiply every limb by the integer c (given as its residues cres[i]) */
void oc_poly_mul_scalar(const u64 *a, const u64 *cres, u64 *out, int nl, int logN, const u64 *m)
{
    u64 N = 1ULL << logN;
    for (int i = 0; i < nl; i++)
        for (u64 j = 0; j < N; j++) out[i * N + j] = mulm(a[i * N + j], cres[i], m[i]);
}

/* Galois automorphism X -> X^g (g odd): coefficient j moves to j*g mod 2N with a
 * sign flip when it lands in [N, 2N) because X^N = -1. */
void oc_automorph(const u64 *a, u64 *out, int nl, int logN, const u64 *m, u64 g)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
#pragma omp parallel for
    for (int i = 0; i < nl; i++)
        for (u64 j = 0; j < N; j++) {
            u64 e = (u64)(((u128)j * g) % twoN);
            u64 v = a[i * N + j];
            if (e < N) out[i * N + e] = v;
            else out[i * N + e - N] = v ? m[i] - v : 0;
        }
}

/*
 * Rescale by the last prime with rounding:
 * c' = round(c / q_l) = (c + h - [c + h]_{q_l}) / q_l with h = floor(q_l / 2).
 * Input (l+1) limbs, output l limbs (coefficient form).
 */
void oc_rescale(const u64 *c, u64 *out, int l, int logN, const u64 *q)
{
    u64 N = 1ULL << logN;
    u64 ql = q[l], h = ql >> 1;
#pragma omp parallel for
    for (int i = 0; i < l; i++) {
        u64 qi = q[i];
        u64 inv = oc_invm(ql % qi, qi), hi = h % qi;
        for (u64 j = 0; j < N; j++) {
            u64 r = (c[(u64)l * N + j] + h) % ql;
            u64 t = subm(r % qi, hi, qi);
            out[i * N + j] = mulm(subm(c[i * N + j], t, qi), inv, qi);
        }
    }
}

/*
 * Fast basis conversion from basis B = {b_0..b_{ns-1}} to C = {c_0..c_{nd-1}}:
 * Conv(x)_p = sum_j [x_j * (B/b_j)^-1]_{b_j} * (B/b_j)  mod p, no overflow
 * correction (the result is x + u*B for a small integer u).
 */
void oc_bconv(const u64 *x, int ns, const u64 *sm, u64 *out, int nd, const u64 *dm, int logN)
{
    u64 N = 1ULL << logN;
    u64 *invhat = malloc(ns * sizeof(u64));
    u64 *hat = malloc((size_t)ns * nd * sizeof(u64));
    for (int j = 0; j < ns; j++) {
        u64 h = 1;
        for (int k = 0; k < ns; k++)
            if (k != j) h = mulm(h, sm[k] % sm[j], sm[j]);
        invhat[j] = oc_invm(h, sm[j]);
        for (int p = 0; p < nd; p++) {
            u64 hp = 1;
            for (int k = 0; k < ns; k++)
                if (k != j) hp = mulm(hp, sm[k] % dm[p], dm[p]);
            hat[j * nd + p] = hp;
        }
    }
#pragma omp parallel
    {
        u64 *y = malloc(ns * sizeof(u64));
#pragma omp for
        for (u64 n = 0; n < N; n++) {
            for (int j = 0; j < ns; j++) y[j] = mulm(x[j * N + n], invhat[j], sm[j]);
            for (int p = 0; p < nd; p++) {
                u64 acc = 0;
                for (int j = 0; j < ns; j++) acc = addm(acc, mulm(y[j], hat[j * nd + p], dm[p]), dm[p]);
                out[p * N + n] = acc;
            }
        }
        free(y);
    }
    free(hat);
    free(invhat);
}

/*
 * ModDown: a over Q_l u P (nq + alpha limbs, Q limbs first) ->
 * (a_Q - Conv_{P->Q}(a_P)) * P^-1  over Q_l.
 */
void oc_moddown(const u64 *a, u64 *out, int nq, int alpha, int logN, const u64 *q, const u64 *p)
{
    u64 N = 1ULL << logN;
    u64 *conv = malloc((size_t)nq * N * sizeof(u64));
    oc_bconv(a + (u64)nq * N, alpha, p, conv, nq, q, logN);
#pragma omp parallel for
    for (int i = 0; i < nq; i++) {
        u64 P = 1;
        for (int k = 0; k < alpha; k++) P = mulm(P, p[k] % q[i], q[i]);
        u64 pinv = oc_invm(P, q[i]);
        for (u64 j = 0; j < N; j++)
            out[i * N + j] = mulm(subm(a[i * N + j], conv[i * N + j], q[i]), pinv, q[i]);
    }
    free(conv);
}

/*
 * Hybrid key switch of d (level l, nq = l+1 limbs, coefficient form).
 * keys: switching key in coefficient form, laid out [dnum_top][2][L+1+alpha][N]
 *       where component 0 is b_j and component 1 is a_j; digit j covers the Q
 *       limbs [j*w, j*w+w).
 * If galois != 0 the automorphism X -> X^galois is applied to every extended
 * digit after ModUp (this is how a rotation is defined here, hoisting-ready).
 * Output (u0, u1) over Q_l, coefficient form:  u0 + u1*s ~= d*s'  (or
 * sigma(d)*s' for rotations).
 */
/* The key switch before its ModDown: acc0, acc1 ([l+1+alpha][N] each, Q_l
 * then P limbs, coefficient form, zeroed by the caller) receive
 * sum_j ext_j * key_j over Q_l u P, ext_j the digit's ModUp with the Galois
 * automorphism applied when galois != 0. */
void oc_keyswitch_acc(const u64 *d, int l, const u64 *keys, int L, int alpha, int w, const u64 *q,
                      const u64 *p, int logN, u64 galois, u64 *acc0, u64 *acc1)
{
    u64 N = 1ULL << logN;
    int nq = l + 1, next = nq + alpha, ktot = L + 1 + alpha;
    int ndig = (nq + w - 1) / w;
    u64 *mods = malloc(next * sizeof(u64));
    for (int i = 0; i < nq; i++) mods[i] = q[i];
    for (int i = 0; i < alpha; i++) mods[nq + i] = p[i];
    u64 *ext = malloc((size_t)next * N * sizeof(u64));
    u64 *tmp = malloc((size_t)next * N * sizeof(u64));
    for (int j = 0; j < ndig; j++) {
        int lo = j * w, hi = lo + w < nq ? lo + w : nq;
        int nsrc = hi - lo;
        /* ModUp: copy the digit's own limbs, convert to every other limb */
        int nt = next - nsrc;
        u64 *tm = malloc(nt * sizeof(u64));
        int *tidx = malloc(nt * sizeof(int));
        int c = 0;
        for (int t = 0; t < next; t++)
            if (t < lo || t >= hi) { tm[c] = mods[t]; tidx[c] = t; c++; }
        u64 *conv = malloc((size_t)nt * N * sizeof(u64));
        oc_bconv(d + (u64)lo * N, nsrc, q + lo, conv, nt, tm, logN);
        for (int t = lo; t < hi; t++) memcpy(ext + (u64)t * N, d + (u64)t * N, N * sizeof(u64));
        for (int k = 0; k < nt; k++) memcpy(ext + (u64)tidx[k] * N, conv + (u64)k * N, N * sizeof(u64));
        free(conv);
        free(tidx);
        free(tm);
        if (galois) {
            oc_automorph(ext, tmp, next, logN, mods, galois);
            memcpy(ext, tmp, (size_t)next * N * sizeof(u64));
        }
        /* inner product with the key digit over every limb of Q_l u P */
#pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < next; t++) {
            int kt = t < nq ? t : L + 1 + (t - nq);
            const u64 *kb = keys + (((u64)j * 2 + 0) * ktot + kt) * N;
            const u64 *ka = keys + (((u64)j * 2 + 1) * ktot + kt) * N;
            u64 *prod = malloc(N * sizeof(u64));
            oc_negacyclic_mul(ext + (u64)t * N, kb, prod, logN, mods[t]);
            for (u64 n = 0; n < N; n++) acc0[t * N + n] = addm(acc0[t * N + n], prod[n], mods[t]);
            oc_negacyclic_mul(ext + (u64)t * N, ka, prod, logN, mods[t]);
            for (u64 n = 0; n < N; n++) acc1[t * N + n] = addm(acc1[t * N + n], prod[n], mods[t]);
            free(prod);
        }
    }
    free(tmp);
    free(ext);
    free(mods);
}

void oc_keyswitch(const u64 *d, int l, const u64 *keys, int L, int alpha, int w, const u64 *q,
                  const u64 *p, int logN, u64 galois, u64 *u0, u64 *u1)
{
    u64 N = 1ULL << logN;
    int nq = l + 1, next = nq + alpha;
    u64 *acc0 = calloc((size_t)next * N, sizeof(u64));
    u64 *acc1 = calloc((size_t)next * N, sizeof(u64));
    oc_keyswitch_acc(d, l, keys, L, alpha, w, q, p, logN, galois, acc0, acc1);
    oc_moddown(acc0, u0, nq, alpha, logN, q, p);
    oc_moddown(acc1, u1, nq, alpha, logN, q, p);
    free(acc1);
    free(acc0);
}

/* ------------------------------------------------------------------------- */
/* ChaCha20 (RFC 8439) and the samplers built on it                             */
/* ------------------------------------------------------------------------- */
static u32 rotl32(u32 x, int n) { return (x << n) | (x >> (32 - n)); }

void oc_chacha_quarter(u32 *a, u32 *b, u32 *c, u32 *d)
{
    *a += *b; *d ^= *a; *d = rotl32(*d, 16);
    *c += *d; *b ^= *c; *b = rotl32(*b, 12);
    *a += *b; *d ^= *a; *d = rotl32(*d, 8);
    *c += *d; *b ^= *c; *b = rotl32(*b, 7);
}

/* block function: key[8], counter, nonce[3] -> out[16] words */
void oc_chacha20_block(const u32 *key, u32 counter, const u32 *nonce, u32 *out)
{
    u32 st[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    for (int i = 0; i < 8; i++) st[4 + i] = key[i];
    st[12] = counter;
    st[13] = nonce[0];
    st[14] = nonce[1];
    st[15] = nonce[2];
    u32 x[16];
    memcpy(x, st, sizeof(x));
    for (int r = 0; r < 10; r++) {
        oc_chacha_quarter(&x[0], &x[4], &x[8], &x[12]);
        oc_chacha_quarter(&x[1], &x[5], &x[9], &x[13]);
        oc_chacha_quarter(&x[2], &x[6], &x[10], &x[14]);
        oc_chacha_quarter(&x[3], &x[7], &x[11], &x[15]);
        oc_chacha_quarter(&x[0], &x[5], &x[10], &x[15]);
        oc_chacha_quarter(&x[1], &x[6], &x[11], &x[12]);
        oc_chacha_quarter(&x[2], &x[7], &x[8], &x[13]);
        oc_chacha_quarter(&x[3], &x[4], &x[9], &x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + st[i];
}

/* a word stream: key from the 64-bit seed, nonce = (purpose, id, sub) */
typedef struct {
    u32 key[8], nonce[3], counter, buf[16];
    int pos;
} stream;

static void stream_init(stream *s, u64 seed, u32 purpose, u32 id, u32 sub)
{
    memset(s, 0, sizeof(*s));
    s->key[0] = (u32)seed;
    s->key[1] = (u32)(seed >> 32);
    s->nonce[0] = purpose;
    s->nonce[1] = id;
    s->nonce[2] = sub;
    s->pos = 16;
}

static u32 next32(stream *s)
{
    if (s->pos == 16) {
        oc_chacha20_block(s->key, s->counter++, s->nonce, s->buf);
        s->pos = 0;
    }
    return s->buf[s->pos++];
}

static u64 next64(stream *s)
{
    u64 lo = next32(s);
    u64 hi = next32(s);
    return lo | (hi << 32);
}

/* uniform residues mod m by rejection on the low bitlen(m) bits */
void oc_sample_uniform(u64 seed, u32 purpose, u32 id, u32 sub, u64 m, int logN, u64 *out)
{
    stream s;
    stream_init(&s, seed, purpose, id, sub);
    int bits = 64 - __builtin_clzll(m);
    u64 mask = bits == 64 ? ~0ULL : ((1ULL << bits) - 1);
    for (u64 j = 0; j < (1ULL << logN); j++) {
        u64 v;
        do v = next64(&s) & mask; while (v >= m);
        out[j] = v;
    }
}

/* uniform ternary {-1,0,1}: two bits, value 3 rejected */
void oc_sample_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int logN, int64_t *out)
{
    stream s;
    stream_init(&s, seed, purpose, id, sub);
    for (u64 j = 0; j < (1ULL << logN); j++) {
        u32 v;
        do v = next32(&s) & 3u; while (v == 3u);
        out[j] = (int64_t)v - 1;
    }
}

/*
 * Sparse ternary secret: exactly h coefficients in {-1, 1}, the others 0.
 * Each 32-bit word w of the stream proposes position w mod N (the low logN
 * bits) with sign w >> 31 (1: -1); a position already taken is skipped.
 * Requires 0 <= h <= N and logN <= 16 (position and sign bits are disjoint).
 */
void oc_sample_sparse_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int logN, int h, int64_t *out)
{
    u64 N = 1ULL << logN;
    memset(out, 0, N * sizeof(int64_t));
    stream s;
    stream_init(&s, seed, purpose, id, sub);
    for (int placed = 0; placed < h;) {
        u32 w = next32(&s);
        u64 pos = w & (N - 1);
        if (out[pos]) continue;
        out[pos] = (w >> 31) ? -1 : 1;
        placed++;
    }
}

/*
 * Rounded Gaussian, sigma given, truncated to |e| <= 19: 39 thresholds
 * T[i] = floor(2^64 * sum_{k<=i-19} rho(k) / sum rho), rho(k) = exp(-k^2/(2 sigma^2)),
 * T[38] = 2^64-1.  A 64-bit word v maps to e = (first i with v < T[i]) - 19.
 */
void oc_gauss_table(double sigma, u64 *T)
{
    double rho[39], total = 0.0, cum = 0.0;
    for (int i = 0; i < 39; i++) {
        int k = i - 19;
        rho[i] = exp(-(double)(k * k) / (2.0 * sigma * sigma));
    }
    for (int i = 0; i < 39; i++) total += rho[i];
    for (int i = 0; i < 38; i++) {
        cum += rho[i];
        T[i] = (u64)ldexp(cum / total, 64);
    }
    T[38] = ~0ULL;
}

void oc_sample_gauss(u64 seed, u32 purpose, u32 id, u32 sub, double sigma, int logN, int64_t *out)
{
    u64 T[39];
    oc_gauss_table(sigma, T);
    stream s;
    stream_init(&s, seed, purpose, id, sub);
    for (u64 j = 0; j < (1ULL << logN); j++) {
        u64 v = next64(&s);
        int i = 0;
        while (i < 38 && v >= T[i]) i++;
        out[j] = (int64_t)i - 19;
    }
}

/* signed small integers -> residues over nl limbs */
void oc_small_to_rns(const int64_t *e, u64 *out, int nl, int logN, const u64 *m)
{
    u64 N = 1ULL << logN;
#pragma omp parallel for
    for (int i = 0; i < nl; i++)
        for (u64 j = 0; j < N; j++) {
            int64_t v = e[j];
            u64 a = (u64)(v < 0 ? -v : v) % m[i];
            out[i * N + j] = (v < 0 && a) ? m[i] - a : a;
        }
}

/* ------------------------------------------------------------------------- */
/* key generation                                                              */
/* ------------------------------------------------------------------------- */
/*
 * Switching key from s' to s, over all L+1+alpha limbs (coefficient form):
 *   b_j = -a_j*s + e_j + [P]_{q_i} * s'  on the Q limbs of digit j,
 *   b_j = -a_j*s + e_j                    on every other limb,
 * a_j uniform from stream (2, key_id, j<<16 | limb), e_j Gaussian from
 * stream (3, key_id, j<<16).
 * s_res, sp_res: residues of s and s' over all L+1+alpha limbs.
 * keys out: [dnum][2][L+1+alpha][N].
 */
void oc_gen_switch_key(u64 seed, u32 key_id, const u64 *s_res, const u64 *sp_res, int L, int alpha,
                       int w, const u64 *q, const u64 *p, int logN, double sigma, u64 *keys)
{
    u64 N = 1ULL << logN;
    int ktot = L + 1 + alpha;
    int dnum = (L + 1 + w - 1) / w;
    u64 *mods = malloc(ktot * sizeof(u64));
    for (int i = 0; i <= L; i++) mods[i] = q[i];
    for (int i = 0; i < alpha; i++) mods[L + 1 + i] = p[i];
    int64_t *e = malloc(N * sizeof(int64_t));
    for (int j = 0; j < dnum; j++) {
        oc_sample_gauss(seed, 3, key_id, (u32)j << 16, sigma, logN, e);
#pragma omp parallel for schedule(dynamic, 1)
        for (int t = 0; t < ktot; t++) {
            u64 *eres = malloc(N * sizeof(u64));
            u64 *as = malloc(N * sizeof(u64));
            u64 m = mods[t];
            u64 *kb = keys + (((u64)j * 2 + 0) * ktot + t) * N;
            u64 *ka = keys + (((u64)j * 2 + 1) * ktot + t) * N;
            oc_sample_uniform(seed, 2, key_id, ((u32)j << 16) | (u32)t, m, logN, ka);
            oc_small_to_rns(e, eres, 1, logN, &m);
            oc_negacyclic_mul(ka, s_res + (u64)t * N, as, logN, m);
            u64 Pm = 0;
            int in_digit = (t <= L) && (t >= j * w) && (t < j * w + w);
            if (in_digit) {
                Pm = 1;
                for (int k = 0; k < alpha; k++) Pm = mulm(Pm, p[k] % m, m);
            }
            for (u64 n = 0; n < N; n++) {
                u64 v = subm(eres[n], as[n], m);
                if (in_digit) v = addm(v, mulm(Pm, sp_res[(u64)t * N + n], m), m);
                kb[n] = v;
            }
            free(as);
            free(eres);
        }
    }
    free(e);
    free(mods);
}

/* ------------------------------------------------------------------------- */
/* double-double arithmetic and the canonical embedding                         */
/* ------------------------------------------------------------------------- */
typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } cdd;

static dd two_sum(double a, double b)
{
    double s = a + b, bb = s - a;
    dd r = {s, (a - (s - bb)) + (b - bb)};
    return r;
}
static dd quick_two_sum(double a, double b)
{
    double s = a + b;
    dd r = {s, b - (s - a)};
    return r;
}
static dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
static dd dd_neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }
static dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
static dd dd_mul(dd a, dd b)
{
    double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p, e);
}
static dd dd_mul_d(dd a, double b)
{
    double p = a.hi * b;
    double e = fma(a.hi, b, -p);
    e += a.lo * b;
    return quick_two_sum(p, e);
}
static dd dd_from(double a) { dd r = {a, 0.0}; return r; }
static dd dd_div_d(dd a, double b)
{
    /* long division: q1 = a/b, remainder, correction */
    double q1 = a.hi / b;
    dd p = dd_mul_d(dd_from(q1), b);
    dd r = dd_sub(a, p);
    double q2 = r.hi / b;
    return quick_two_sum(q1, q2);
}

static cdd cdd_add(cdd a, cdd b) { cdd r = {dd_add(a.re, b.re), dd_add(a.im, b.im)}; return r; }
static cdd cdd_sub(cdd a, cdd b) { cdd r = {dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; return r; }
static cdd cdd_mul(cdd a, cdd b)
{
    cdd r = {dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)),
             dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
    return r;
}

/* pi in double-double */
static const dd DD_PI = {3.141592653589793116e+00, 1.224646799147353207e-16};

/* sin and cos of x (|x| <= pi/4) by Taylor series in double-double */
static void dd_sincos_small(dd x, dd *s, dd *c)
{
    dd x2 = dd_mul(x, x);
    dd term = x, sum = x;
    for (int n = 1; n <= 16; n++) {
        term = dd_mul(term, x2);
        term = dd_div_d(term, (double)((2 * n) * (2 * n + 1)));
        sum = (n & 1) ? dd_sub(sum, term) : dd_add(sum, term);
    }
    *s = sum;
    term = dd_from(1.0);
    sum = term;
    for (int n = 1; n <= 16; n++) {
        term = dd_mul(term, x2);
        term = dd_div_d(term, (double)((2 * n - 1) * (2 * n)));
        sum = (n & 1) ? dd_sub(sum, term) : dd_add(sum, term);
    }
    *c = sum;
}

/* zeta^e with zeta = exp(i*pi/N), e taken mod 2N */
static cdd root_pow(u64 e, u64 N)
{
    e %= 2 * N;
    int neg = 0;
    if (e >= N) { e -= N; neg = 1; }              /* zeta^N = -1           */
    int quarter = 0;
    if (e >= N / 2) { e -= N / 2; quarter = 1; }  /* zeta^(N/2) = i        */
    dd s, c;
    if (e <= N / 4) {
        dd th = dd_mul_d(DD_PI, (double)e / (double)N);
        dd_sincos_small(th, &s, &c);
    } else {
        dd th = dd_mul_d(DD_PI, (double)(N / 2 - e) / (double)N);
        dd_sincos_small(th, &c, &s);              /* cos/sin swap at pi/2 - th */
    }
    cdd r = {c, s};
    if (quarter) { cdd t = {dd_neg(r.im), r.re}; r = t; }
    if (neg) { r.re = dd_neg(r.re); r.im = dd_neg(r.im); }
    return r;
}

/* in-place radix-2 DFT: X_k = sum_j x_j * zeta^(sgn * 2 j k) */
static void cdd_dft(cdd *x, u64 N, int sgn, const cdd *roots /* zeta^e, e<2N */)
{
    for (u64 i = 1, j = 0; i < N; i++) {
        u64 bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cdd t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (u64 len = 2; len <= N; len <<= 1) {
        u64 half = len >> 1, step = N / len;
        for (u64 i = 0; i < N; i += len)
            for (u64 j = 0; j < half; j++) {
                u64 e = (2 * j * step) % (2 * N);
                if (sgn < 0) e = (2 * N - e) % (2 * N);
                cdd v = cdd_mul(x[i + j + half], roots[e]);
                cdd u = x[i + j];
                x[i + j] = cdd_add(u, v);
                x[i + j + half] = cdd_sub(u, v);
            }
    }
}

static cdd *make_roots(u64 N)
{
    cdd *r = malloc(2 * N * sizeof(cdd));
    for (u64 e = 0; e < 2 * N; e++) r[e] = root_pow(e, N);
    return r;
}

/* round a double-double to the nearest integer, ties to even.  v.hi - r is
 * exact (Sterbenz), so v = r + d.hi + d.lo exactly; g is the exact fraction of
 * d.hi and |d.lo| is below half an ulp of d.hi. */
static i128 dd_round(dd v)
{
    double r = nearbyint(v.hi);
    dd d = two_sum(v.hi - r, v.lo);
    double f = floor(d.hi);
    double g = d.hi - f;
    i128 n = (i128)r + (i128)f;
    if (g > 0.5 || (g == 0.5 && d.lo > 0)) n += 1;
    else if (g == 0.5 && d.lo == 0 && (n & 1)) n += 1;
    return n;
}

void oc_encode_c(const double *re, const double *im, int nz, double scale, int logN, const u64 *m, int nl,
                 u64 *out);

/*
 * Encode real slot values z[0..nz) (the remaining of the N/2 slots are 0) at
 * scale `scale`: m(X) = round(scale * tau^-1(z)), with slot j <-> root
 * zeta^(5^j) and its conjugate zeta^(-5^j).  Output residues over nl limbs.
 */
void oc_encode(const double *z, int nz, double scale, int logN, const u64 *m, int nl, u64 *out)
{
    oc_encode_c(z, NULL, nz, scale, logN, m, nl, out);
}

/* Complex slots z_j = re[j] + i im[j] (im may be NULL: real slots): the value
 * at root zeta^(5^j) is z_j and at its conjugate root conj(z_j), so the
 * coefficients are real. */
void oc_encode_c(const double *re, const double *im, int nz, double scale, int logN, const u64 *m, int nl,
                 u64 *out)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    cdd *roots = make_roots(N);
    cdd *A = calloc(N, sizeof(cdd));
    u64 e = 1;
    for (u64 j = 0; j < N / 2; j++) {
        double v = j < (u64)nz ? re[j] : 0.0;
        double w = (im && j < (u64)nz) ? im[j] : 0.0;
        u64 k = (e - 1) / 2, kc = (twoN - e - 1) / 2;
        A[k].re = dd_from(v);
        A[k].im = dd_from(w);
        A[kc].re = dd_from(v);
        A[kc].im = dd_from(-w);
        e = (e * 5) % twoN;
    }
    /* B_i = sum_k A_k omega^(-ik),  m_i = Re(B_i zeta^-i) * scale / N */
    cdd_dft(A, N, -1, roots);
    double sc = scale / (double)N;
    for (u64 i = 0; i < N; i++) {
        cdd zi = roots[(twoN - i) % twoN];
        dd re = dd_sub(dd_mul(A[i].re, zi.re), dd_mul(A[i].im, zi.im));
        i128 c = dd_round(dd_mul_d(re, sc));
        for (int t = 0; t < nl; t++) {
            u128 a = (u128)(c < 0 ? -c : c) % m[t];
            u64 r = (u64)a;
            out[t * N + i] = (c < 0 && r) ? m[t] - r : r;
        }
    }
    free(A);
    free(roots);
}

/* the coefficient the encoder produces for a constant c: round(c * scale), the
 * exact product rounded ties-to-even; returned as residues over nl limbs */
void oc_encode_const(double c, double scale, const u64 *m, int nl, u64 *out)
{
    double p = c * scale;
    dd v = {p, fma(c, scale, -p)};
    i128 r = dd_round(v);
    for (int t = 0; t < nl; t++) {
        u128 a = (u128)(r < 0 ? -r : r) % m[t];
        u64 x = (u64)a;
        out[t] = (r < 0 && x) ? m[t] - x : x;
    }
}

/* integer coefficient of the encoder, for tests: coefficients as two int64
 * halves would be awkward, so expose the rounded value as a double pair */
void oc_encode_coeffs_dd(const double *z, int nz, double scale, int logN, double *hi, double *lo)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    cdd *roots = make_roots(N);
    cdd *A = calloc(N, sizeof(cdd));
    u64 e = 1;
    for (u64 j = 0; j < N / 2; j++) {
        double v = j < (u64)nz ? z[j] : 0.0;
        A[(e - 1) / 2].re = dd_from(v);
        A[(twoN - e - 1) / 2].re = dd_from(v);
        e = (e * 5) % twoN;
    }
    cdd_dft(A, N, -1, roots);
    double sc = scale / (double)N;
    for (u64 i = 0; i < N; i++) {
        cdd zi = roots[(twoN - i) % twoN];
        dd re = dd_mul_d(dd_sub(dd_mul(A[i].re, zi.re), dd_mul(A[i].im, zi.im)), sc);
        hi[i] = re.hi;
        lo[i] = re.lo;
    }
    free(A);
    free(roots);
}

/*
 * Decode: centered coefficients of one limb modulo q0 (|m_i| < q0/2) ->
 * slot values z_j = m(zeta^(5^j)) / scale for j < nz (real part).
 */
void oc_decode(const u64 *c, u64 q0, double scale, int logN, int nz, double *z)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    cdd *roots = make_roots(N);
    cdd *A = calloc(N, sizeof(cdd));
    for (u64 i = 0; i < N; i++) {
        int64_t v = c[i] > q0 / 2 ? -(int64_t)(q0 - c[i]) : (int64_t)c[i];
        double hi = (double)v;
        double lo = (double)(v - (int64_t)hi);
        dd m = {hi, lo};
        cdd zi = roots[i];
        A[i].re = dd_mul(m, zi.re);
        A[i].im = dd_mul(m, zi.im);
    }
    cdd_dft(A, N, +1, roots);
    u64 e = 1;
    for (int j = 0; j < nz; j++) {
        dd v = A[(e - 1) / 2].re;
        z[j] = (v.hi + v.lo) / scale;
        e = (e * 5) % twoN;
    }
    free(A);
    free(roots);
}

/* direct O(N) evaluation of one encoder coefficient (before rounding), used to
 * pin the FFT: (2*scale/N) * sum_j z_j cos(pi * (i*5^j mod 2N) / N) */
double oc_encode_coeff_direct(const double *z, int nz, double scale, int logN, u64 i)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    dd acc = dd_from(0.0);
    u64 e = 1;
    for (u64 j = 0; j < N / 2; j++) {
        double v = j < (u64)nz ? z[j] : 0.0;
        u64 ang = (u64)(((u128)i * e) % twoN);
        cdd r = root_pow(ang, N);
        acc = dd_add(acc, dd_mul_d(r.re, v));
        e = (e * 5) % twoN;
    }
    acc = dd_mul_d(acc, 2.0 * scale / (double)N);
    return acc.hi + acc.lo;
}

/* Decode to complex slots: re[j] + i im[j] = m(zeta^(5^j)) / scale, j < nz. */
void oc_decode_c(const u64 *c, u64 q0, double scale, int logN, int nz, double *re, double *im)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    cdd *roots = make_roots(N);
    cdd *A = calloc(N, sizeof(cdd));
    for (u64 i = 0; i < N; i++) {
        int64_t v = c[i] > q0 / 2 ? -(int64_t)(q0 - c[i]) : (int64_t)c[i];
        double hi = (double)v;
        double lo = (double)(v - (int64_t)hi);
        dd m = {hi, lo};
        A[i].re = dd_mul(m, roots[i].re);
        A[i].im = dd_mul(m, roots[i].im);
    }
    cdd_dft(A, N, +1, roots);
    u64 e = 1;
    for (int j = 0; j < nz; j++) {
        cdd v = A[(e - 1) / 2];
        re[j] = (v.re.hi + v.re.lo) / scale;
        im[j] = (v.im.hi + v.im.lo) / scale;
        e = (e * 5) % twoN;
    }
    free(A);
    free(roots);
}

/* zeta^e (zeta = exp(i pi / N)) for every e < 2N, each part rounded to the
 * nearest double (from its double-double value). */
void oc_root_table(int logN, double *re, double *im)
{
    u64 N = 1ULL << logN;
    for (u64 e = 0; e < 2 * N; e++) {
        cdd r = root_pow(e, N);
        re[e] = r.re.hi + r.re.lo;
        im[e] = r.im.hi + r.im.lo;
    }
}

/* direct O(N) evaluation of one encoder coefficient for complex slots:
 * (2 scale / N) sum_j (re_j cos(pi a_j / N) + im_j sin(pi a_j / N)),
 * a_j = i 5^j mod 2N (the real part of (2/N) sum_j z_j zeta^(-i 5^j)) */
double oc_encode_coeff_direct_c(const double *re, const double *im, int nz, double scale, int logN, u64 i)
{
    u64 N = 1ULL << logN, twoN = 2 * N;
    dd acc = dd_from(0.0);
    u64 e = 1;
    for (u64 j = 0; j < N / 2; j++) {
        if (j < (u64)nz) {
            u64 ang = (u64)(((u128)i * e) % twoN);
            cdd r = root_pow(ang, N);
            acc = dd_add(acc, dd_mul_d(r.re, re[j]));
            acc = dd_add(acc, dd_mul_d(r.im, im[j]));
        }
        e = (e * 5) % twoN;
    }
    acc = dd_mul_d(acc, 2.0 * scale / (double)N);
    return acc.hi + acc.lo;
}
