// Host-side number theory, ChaCha20 sampling and the canonical-embedding
// encoder of the GPU library (client side and offline model compile).
#include "hostmath.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

namespace hk {

// ------------------------------------------------------------- number theory
u64 hpow(u64 a, u64 e, u64 q)
{
    u64 r = 1 % q, b = a % q;
    for (; e; e >>= 1, b = hmul(b, b, q))
        if (e & 1) r = hmul(r, b, q);
    return r;
}

u64 hinv(u64 a, u64 q)
{
    // extended Euclid on signed 128-bit integers
    i128 t = 0, nt = 1, r = q, nr = a % q;
    while (nr != 0) {
        i128 k = r / nr;
        i128 tmp = t - k * nt;
        t = nt;
        nt = tmp;
        tmp = r - k * nr;
        r = nr;
        nr = tmp;
    }
    if (r != 1) throw std::runtime_error("hinv: not invertible");
    if (t < 0) t += q;
    return (u64)t;
}

bool is_prime64(u64 n)
{
    if (n < 2) return false;
    const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : small) {
        if (n == p) return true;
        if (n % p == 0) return false;
    }
    u64 d = n - 1;
    int r = __builtin_ctzll(d);
    d >>= r;
    for (u64 a : small) {
        u64 x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int i = 1; i < r && witness; i++) {
            x = hmul(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

static bool used_before(const std::vector<u64> &v, u64 c)
{
    for (u64 x : v)
        if (x == c) return true;
    return false;
}

void make_chain(int logN, int base_bits, int L, int scale_bits, int alpha, int special_bits, int boot_levels,
                int boot_bits, std::vector<u64> &q, std::vector<u64> &p, std::vector<double> &S)
{
    const u64 M = 2ull << logN;
    std::vector<u64> used;
    q.assign(L + 1, 0);
    p.assign(alpha, 0);
    S.assign(L + 1, 0.0);
    // q_0: largest prime = 1 mod 2N below 2^base_bits
    u64 c = ((1ull << base_bits) - 2) / M * M + 1;
    while (!is_prime64(c)) c -= M;
    q[0] = c;
    used.push_back(c);
    // special primes: descending below 2^special_bits, skipping used ones
    c = ((1ull << special_bits) - 2) / M * M + 1;
    for (int i = 0; i < alpha; i++) {
        while (!is_prime64(c) || used_before(used, c)) c -= M;
        p[i] = c;
        used.push_back(c);
        c -= M;
    }
    // scale primes top-down keeping the canonical scale near Delta_l: the
    // top boot_levels levels (those a bootstrapping consumes) near
    // 2^boot_bits, the computation levels below near 2^scale_bits, whose
    // top level takes S = 2^scale_bits
    const int top_c = L - boot_levels;
    double s = std::ldexp(1.0, boot_levels > 0 ? boot_bits : scale_bits);
    S[L] = s;
    for (int l = L; l >= 1; l--) {
        const double delta = std::ldexp(1.0, l > top_c ? boot_bits : scale_bits);
        const double target = (s * s) / delta;
        u64 below = (u64)std::floor((target - 1.0) / (double)M) * M + 1;  // <= target
        u64 above = below + M;
        u64 pick = 0;
        while (!pick) {
            double db = target - (double)below, da = (double)above - target;
            if (db <= da) {
                if (is_prime64(below) && !used_before(used, below)) pick = below;
                else below -= M;
            } else {
                if (is_prime64(above) && !used_before(used, above)) pick = above;
                else above += M;
            }
        }
        q[l] = pick;
        used.push_back(pick);
        s = (boot_levels > 0 && l == top_c + 1) ? std::ldexp(1.0, scale_bits) : (s * s) / (double)pick;
        S[l - 1] = s;
    }
}

u64 primitive_2n_root(u64 q, int logN)
{
    const u64 N = 1ull << logN;
    for (u64 x = 2;; x++) {
        u64 r = hpow(x, (q - 1) / (2 * N), q);
        if (hpow(r, N, q) == q - 1) return r;
    }
}

// ------------------------------------------------------------------ ChaCha20
static inline u32 rol(u32 v, int c) { return (v << c) | (v >> (32 - c)); }
#define CHACHA_QR(a, b, c, d)                                                        \
    a += b; d ^= a; d = rol(d, 16); c += d; b ^= c; b = rol(b, 12);                 \
    a += b; d ^= a; d = rol(d, 8);  c += d; b ^= c; b = rol(b, 7);

void chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3], u32 out[16])
{
    u32 in[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, key[0], key[1], key[2], key[3],
                  key[4],      key[5],      key[6],      key[7],      counter, nonce[0], nonce[1], nonce[2]};
    u32 x[16];
    std::memcpy(x, in, sizeof(x));
    for (int i = 0; i < 10; i++) {
        CHACHA_QR(x[0], x[4], x[8], x[12]);
        CHACHA_QR(x[1], x[5], x[9], x[13]);
        CHACHA_QR(x[2], x[6], x[10], x[14]);
        CHACHA_QR(x[3], x[7], x[11], x[15]);
        CHACHA_QR(x[0], x[5], x[10], x[15]);
        CHACHA_QR(x[1], x[6], x[11], x[12]);
        CHACHA_QR(x[2], x[7], x[8], x[13]);
        CHACHA_QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + in[i];
}

ChaChaStream::ChaChaStream(u64 seed, u32 purpose, u32 id, u32 sub) : counter(0), pos(16)
{
    std::memset(key, 0, sizeof(key));
    key[0] = (u32)(seed & 0xffffffffu);
    key[1] = (u32)(seed >> 32);
    nonce[0] = purpose;
    nonce[1] = id;
    nonce[2] = sub;
}

u32 ChaChaStream::next32()
{
    if (pos == 16) {
        chacha20_block(key, counter, nonce, buf);
        counter++;
        pos = 0;
    }
    return buf[pos++];
}

u64 ChaChaStream::next64()
{
    u64 lo = next32();
    return lo | ((u64)next32() << 32);
}

void sample_uniform(u64 seed, u32 purpose, u32 id, u32 sub, u64 q, int N, u64 *out)
{
    ChaChaStream st(seed, purpose, id, sub);
    int nb = 64 - __builtin_clzll(q);
    u64 mask = nb >= 64 ? ~0ull : (1ull << nb) - 1;
    for (int i = 0; i < N; i++) {
        u64 v = st.next64() & mask;
        while (v >= q) v = st.next64() & mask;
        out[i] = v;
    }
}

void sample_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int N, int64_t *out)
{
    ChaChaStream st(seed, purpose, id, sub);
    for (int i = 0; i < N; i++) {
        u32 v = st.next32() & 3u;
        while (v == 3u) v = st.next32() & 3u;
        out[i] = (int64_t)v - 1;
    }
}

// exactly h coefficients in {-1, 1}: each word w proposes position w mod N
// with sign w >> 31 (1: -1); taken positions are skipped
void sample_sparse_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int N, int h, int64_t *out)
{
    if (h < 0 || h > N || N > (1 << 16)) throw std::runtime_error("sparse secret: bad Hamming weight");
    ChaChaStream st(seed, purpose, id, sub);
    std::fill(out, out + N, (int64_t)0);
    for (int placed = 0; placed < h;) {
        const u32 w = st.next32();
        const u32 pos = w & (u32)(N - 1);
        if (out[pos]) continue;
        out[pos] = (w >> 31) ? -1 : 1;
        placed++;
    }
}

void gauss_thresholds(double sigma, u64 T[39])
{
    double w[39];
    for (int k = -19; k <= 19; k++) w[k + 19] = std::exp(-(double)(k * k) / (2.0 * sigma * sigma));
    double sum = 0.0;
    for (int i = 0; i < 39; i++) sum += w[i];
    double run = 0.0;
    for (int i = 0; i < 38; i++) {
        run += w[i];
        T[i] = (u64)std::ldexp(run / sum, 64);
    }
    T[38] = ~0ull;
}

void sample_gauss(u64 seed, u32 purpose, u32 id, u32 sub, double sigma, int N, int64_t *out)
{
    u64 T[39];
    gauss_thresholds(sigma, T);
    ChaChaStream st(seed, purpose, id, sub);
    for (int i = 0; i < N; i++) {
        u64 v = st.next64();
        int k = 0;
        while (k < 38 && v >= T[k]) k++;
        out[i] = k - 19;
    }
}

// ------------------------------------------------------- double-double values
namespace {
struct DD {
    double hi, lo;
};
inline DD dd_two_sum(double a, double b)
{
    double s = a + b;
    double v = s - a;
    return {s, (a - (s - v)) + (b - v)};
}
inline DD dd_fast(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}
inline DD operator+(DD a, DD b)
{
    DD s = dd_two_sum(a.hi, b.hi);
    DD t = dd_two_sum(a.lo, b.lo);
    s = dd_fast(s.hi, s.lo + t.hi);
    return dd_fast(s.hi, s.lo + t.lo);
}
inline DD operator-(DD a) { return {-a.hi, -a.lo}; }
inline DD operator-(DD a, DD b) { return a + (-b); }
inline DD operator*(DD a, DD b)
{
    double p = a.hi * b.hi;
    double e = std::fma(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
    return dd_fast(p, e);
}
inline DD operator*(DD a, double b)
{
    double p = a.hi * b;
    return dd_fast(p, std::fma(a.hi, b, -p) + a.lo * b);
}
inline DD dd_div(DD a, double b)
{
    double q1 = a.hi / b;
    DD r = a - DD{q1, 0.0} * b;
    return dd_fast(q1, r.hi / b);
}
struct CDD {
    DD re, im;
};
inline CDD operator+(CDD a, CDD b) { return {a.re + b.re, a.im + b.im}; }
inline CDD operator-(CDD a, CDD b) { return {a.re - b.re, a.im - b.im}; }
inline CDD operator*(CDD a, CDD b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

const DD PI_DD = {3.141592653589793116e+00, 1.224646799147353207e-16};

// sin and cos of x in [0, pi/4] in double-double: Horner on the Taylor series
void dd_sin_cos(DD x, DD &s, DD &c)
{
    DD x2 = x * x;
    const int K = 17;
    // sin x = x (1 - x^2/(2 3) (1 - x^2/(4 5) (1 - ...)))
    DD ps = {1.0, 0.0};
    for (int k = K; k >= 1; k--) ps = DD{1.0, 0.0} - dd_div(x2 * ps, (double)((2 * k) * (2 * k + 1)));
    s = x * ps;
    DD pc = {1.0, 0.0};
    for (int k = K; k >= 1; k--) pc = DD{1.0, 0.0} - dd_div(x2 * pc, (double)((2 * k - 1) * (2 * k)));
    c = pc;
}

// exp(i pi e / N) for integer e
CDD zeta_pow(long e, long N)
{
    long twoN = 2 * N;
    e %= twoN;
    if (e < 0) e += twoN;
    // write e = quadrant * (N/2) + f, f in [0, N/2)
    long quad = e / (N / 2), f = e % (N / 2);
    DD s, c;
    if (2 * f <= N / 2) {
        dd_sin_cos(PI_DD * ((double)f / (double)N), s, c);
    } else {
        DD s2, c2;
        dd_sin_cos(PI_DD * ((double)(N / 2 - f) / (double)N), s2, c2);
        s = c2;
        c = s2;
    }
    CDD r = {c, s};
    for (long k = 0; k < quad; k++) r = CDD{-r.im, r.re};  // multiply by i
    return r;
}

i128 round_even(DD v)
{
    double fl = std::floor(v.hi);
    DD fr = dd_two_sum(v.hi - fl, v.lo);
    double f2 = std::floor(fr.hi);
    double g = fr.hi - f2;
    i128 base = (i128)fl + (i128)f2;
    if (g > 0.5) return base + 1;
    if (g < 0.5) return base;
    if (fr.lo > 0) return base + 1;
    if (fr.lo < 0) return base;
    return (base & 1) ? base + 1 : base;
}

void put_residues(i128 v, const u64 *mods, int nl, u64 *out, long stride)
{
    u128 mag = (u128)(v < 0 ? -v : v);
    for (int t = 0; t < nl; t++) {
        u64 r = (u64)(mag % mods[t]);
        out[t * stride] = (v < 0 && r) ? mods[t] - r : r;
    }
}
}  // namespace

// The encoder's double-double tables for one ring degree: the FFT twiddles
// zeta^(-4 r) (r < M/2), the final factors zeta^(-i) (i < M) and the
// bit-reversal of the M-point FFT.  Built once per degree (the series that
// give each entry dominate an encode's cost) and kept for the process.
struct EncTables {
    std::vector<CDD> tw, zinv;
    std::vector<long> brv;
};

static const EncTables &enc_tables(int logN)
{
    static std::mutex mu;
    static std::map<int, std::unique_ptr<EncTables>> cache;
    std::lock_guard<std::mutex> lk(mu);
    std::unique_ptr<EncTables> &t = cache[logN];
    if (!t) {
        const long N = 1l << logN, M = N / 2;
        t.reset(new EncTables());
        t->tw.resize(M / 2 > 0 ? M / 2 : 1);
        for (long r = 0; r < M / 2; r++) t->tw[r] = zeta_pow(-4 * r, N);
        t->zinv.resize(M);
        for (long i = 0; i < M; i++) t->zinv[i] = zeta_pow(-i, N);
        int lm = 0;
        while ((1l << lm) < M) lm++;
        t->brv.resize(M);
        for (long i = 0; i < M; i++) {
            long src = 0;
            for (int b = 0; b < lm; b++)
                if (i >> b & 1) src |= 1l << (lm - 1 - b);
            t->brv[i] = src;
        }
    }
    return *t;
}

void encode_rns(const double *z, size_t n, double scale, int logN, const u64 *mods, int nl, u64 *out)
{
    encode_rns_c(z, nullptr, n, scale, logN, mods, nl, out);
}

void encode_rns_c(const double *re, const double *im, size_t n, double scale, int logN, const u64 *mods, int nl,
                  u64 *out)
{
    const long N = 1l << logN, M = N / 2, twoN = 2 * N;
    if ((long)n > M) throw std::runtime_error("encode: too many slots");
    const EncTables &T = enc_tables(logN);
    // w_k = z_j where 5^j = 4k + 1 (mod 2N); the values at the conjugate
    // roots are the conjugates, so only these M enter (see below)
    std::vector<CDD> w(M, CDD{{0, 0}, {0, 0}});
    long e = 1;
    for (long j = 0; j < M; j++) {
        if ((size_t)j < n) w[(e - 1) / 4] = CDD{DD{re[j], 0.0}, DD{im ? im[j] : 0.0, 0.0}};
        e = e * 5 % twoN;
    }
    // in-place iterative radix-2 DIF with twiddles omega^-r, omega = zeta^4,
    // natural order in, bit-reversed out
    const std::vector<CDD> &tw = T.tw;
    for (long len = M; len >= 2; len >>= 1) {
        long half = len / 2, step = M / len;
        for (long b = 0; b < M; b += len)
            for (long j = 0; j < half; j++) {
                CDD u = w[b + j], v = w[b + j + half];
                w[b + j] = u + v;
                w[b + j + half] = (u - v) * tw[j * step];
            }
    }
    // u_i = (2/N) zeta^-i W_i,  m_i = Re u_i * scale,  m_{i+M} = Im u_i * scale
    const double f = 2.0 * scale / (double)N;
    for (long i = 0; i < M; i++) {
        CDD u = w[T.brv[i]] * T.zinv[i];
        put_residues(round_even(u.re * f), mods, nl, out + i, N);
        put_residues(round_even(u.im * f), mods, nl, out + i + M, N);
    }
}

void zeta_table(int logN, double *re, double *im)
{
    const long N = 1l << logN;
    for (long e = 0; e < 2 * N; e++) {
        const CDD r = zeta_pow(e, N);
        re[e] = r.re.hi + r.re.lo;
        im[e] = r.im.hi + r.im.lo;
    }
}

void encode_const_rns(double c, double scale, const u64 *mods, int nl, u64 *out)
{
    double p = c * scale;
    put_residues(round_even(DD{p, std::fma(c, scale, -p)}), mods, nl, out, 1);
}

void decode_limb(const u64 *coef, u64 q0, double scale, int logN, size_t n, double *z)
{
    const long N = 1l << logN, M = N / 2, twoN = 2 * N;
    typedef std::complex<double> cd;
    std::vector<cd> u(M);
    auto centred = [&](u64 v) { return v > q0 / 2 ? -(double)(q0 - v) : (double)v; };
    for (long i = 0; i < M; i++) {
        double ang = M_PI * (double)i / (double)N;
        u[i] = cd(centred(coef[i]), centred(coef[i + M])) * cd(std::cos(ang), std::sin(ang));
    }
    // forward DFT of length M: U_k = sum_i u_i omega^{k i}, radix-2 DIF
    for (long len = M; len >= 2; len >>= 1) {
        long half = len / 2, step = M / len;
        for (long b = 0; b < M; b += len)
            for (long j = 0; j < half; j++) {
                double ang = 2.0 * M_PI * (double)(j * step) / (double)M;
                cd u0 = u[b + j], v0 = u[b + j + half];
                u[b + j] = u0 + v0;
                u[b + j + half] = (u0 - v0) * cd(std::cos(ang), std::sin(ang));
            }
    }
    int lm = 0;
    while ((1l << lm) < M) lm++;
    long e = 1;
    for (size_t j = 0; j < n; j++) {
        long k = (e - 1) / 4;
        long src = 0;
        for (int b = 0; b < lm; b++)
            if (k >> b & 1) src |= 1l << (lm - 1 - b);
        z[j] = u[src].real() / scale;
        e = e * 5 % twoN;
    }
}

}  // namespace hk
