// Host-side number theory, sampling and the canonical-embedding encoder.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hk {

typedef unsigned long long u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;
typedef __int128 i128;

inline u64 hmul(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
u64 hpow(u64 a, u64 e, u64 q);
u64 hinv(u64 a, u64 q);        // inverse mod q (extended Euclid)
bool is_prime64(u64 n);
inline u64 shoup_of(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// Prime chain (see hekan.h): q[0..L], p[0..alpha-1], canonical scales S[0..L];
// the top boot_levels primes have boot_bits
void make_chain(int logN, int base_bits, int L, int scale_bits, int alpha, int special_bits, int boot_levels,
                int boot_bits, std::vector<u64> &q, std::vector<u64> &p, std::vector<double> &S);
u64 primitive_2n_root(u64 q, int logN);

// ChaCha20 word stream keyed by a 64-bit seed, nonce (purpose, id, sub)
struct ChaChaStream {
    u32 key[8], nonce[3], counter, buf[16];
    int pos;
    ChaChaStream(u64 seed, u32 purpose, u32 id, u32 sub);
    u32 next32();
    u64 next64();
};
void chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3], u32 out[16]);

void sample_uniform(u64 seed, u32 purpose, u32 id, u32 sub, u64 q, int N, u64 *out);
void sample_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int N, int64_t *out);
void sample_sparse_ternary(u64 seed, u32 purpose, u32 id, u32 sub, int N, int h, int64_t *out);
void gauss_thresholds(double sigma, u64 T[39]);
void sample_gauss(u64 seed, u32 purpose, u32 id, u32 sub, double sigma, int N, int64_t *out);

// Encoder: real slots z[0..n) (rest 0) at `scale` -> integer coefficients
// round(scale * tau^-1(z)) (ties to even), written as residues mod each of
// mods[0..nl) into out[nl][N].
void encode_rns(const double *z, size_t n, double scale, int logN, const u64 *mods, int nl, u64 *out);
// complex slots re[j] + i im[j] (im may be null)
void encode_rns_c(const double *re, const double *im, size_t n, double scale, int logN, const u64 *mods, int nl,
                  u64 *out);
// the doubles nearest the parts of zeta^e = exp(i pi e / N), e < 2N
void zeta_table(int logN, double *re, double *im);
// the constant c: one coefficient round(c * scale) as residues
void encode_const_rns(double c, double scale, const u64 *mods, int nl, u64 *out);
// decode centred coefficients (one limb mod q0) to the first n slots
void decode_limb(const u64 *coef, u64 q0, double scale, int logN, size_t n, double *z);

}  // namespace hk
