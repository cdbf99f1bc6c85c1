// Host-side entry points into the library's bootstrapping and encoder code
// for CPU tests: plain C wrappers around the C++ functions the library runs
// on the host (no device call is made).
#include <cstring>
#include <vector>

#include "../../paper_2409_07751_amd/csrc/boot.hpp"
#include "../../paper_2409_07751_amd/csrc/hostmath.hpp"

extern "C" {

void bh_zeta_table(int logN, double *re, double *im) { hk::zeta_table(logN, re, im); }

void bh_encode_c(const double *re, const double *im, size_t n, double scale, int logN, const uint64_t *mods, int nl,
                 uint64_t *out)
{
    hk::encode_rns_c(re, im, n, scale, logN, reinterpret_cast<const hk::u64 *>(mods), nl,
                     reinterpret_cast<hk::u64 *>(out));
}

// the group's offsets (ascending) into offs (cap entries), its diagonals into
// re/im ([offset index][N/2]); returns the number of offsets, b1 in *b1
int bh_group(int logN, const int *stages, int n, int inverse, long *offs, double *re, double *im, int cap, long *b1)
{
    std::vector<double> zr(2l << logN), zi(2l << logN);
    hk::zeta_table(logN, zr.data(), zi.data());
    hk::BootGroup G = hk::boot_group(logN, std::vector<int>(stages, stages + n), inverse != 0, zr, zi);
    const long M = 1l << (logN - 1);
    int k = 0;
    for (auto &kv : G.diag) {
        if (k < cap) {
            offs[k] = kv.first;
            std::memcpy(re + (size_t)k * M, kv.second.first.data(), M * sizeof(double));
            std::memcpy(im + (size_t)k * M, kv.second.second.data(), M * sizeof(double));
        }
        k++;
    }
    *b1 = G.b1;
    return k;
}

void bh_chain(int logN, int base_bits, int L, int scale_bits, int alpha, int special_bits, int boot_levels,
              int boot_bits, uint64_t *q, uint64_t *p, double *S)
{
    std::vector<hk::u64> qq, pp;
    std::vector<double> ss;
    hk::make_chain(logN, base_bits, L, scale_bits, alpha, special_bits, boot_levels, boot_bits, qq, pp, ss);
    for (size_t i = 0; i < qq.size(); i++) q[i] = qq[i];
    for (size_t i = 0; i < pp.size(); i++) p[i] = pp[i];
    for (size_t i = 0; i < ss.size(); i++) S[i] = ss[i];
}

void bh_sparse(uint64_t seed, int N, int h, int64_t *out) { hk::sample_sparse_ternary(seed, 1, 0, 0, N, h, out); }
}
