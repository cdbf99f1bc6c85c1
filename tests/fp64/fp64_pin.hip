// Host-side harness for the CPU pins of the product's exact FP64 residue
// arithmetic: it calls the very helpers the GPU kernels use (u2d, d2u_mod,
// mulm_fp from the package's modarith.hpp, host-callable) and runs one
// forward negacyclic transform with the GPU path's butterfly arithmetic:
// x_lo, x_hi <- a + r, a - r with r = mulm_fp(x_hi, w, w/q, q) and no
// reduction inside the transform; the stages of the column pass take their
// twiddle from the table (w, w/q), the last eight stages (the row pass over
// 256-word rows) form it as W = mulm_fp(A, B, B/q, q) from a per-row factor A
// and a per-stage factor B with quotient constant W fl(1/q); the output is
// reduced by d2u_mod.  Test infrastructure: built and loaded by
// tests/test_fp64_pins.py only.
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../paper_2409_07751_amd/csrc/modarith.hpp"

using hk::u64;

extern "C" {

void fp_mulm(const double *y, const double *w, const double *c, double q, double *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = hk::mulm_fp(y[i], w[i], c[i], q);
}

void fp_d2u_mod(const double *v, double q, double qi, uint64_t *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = hk::d2u_mod(v[i], q, qi);
}

void fp_u2d(const uint64_t *v, double *out, size_t n)
{
    for (size_t i = 0; i < n; i++) out[i] = hk::u2d(v[i]);
}

// x: N doubles (integers, |x| < 4q) transformed in place in the GPU's
// output order (slot k holds the evaluation at psi^(2 brv(k) + 1)), then
// reduced into out[0, N).  fw[k] = psi^brv(k) mod q (k < N); A, B: the row
// pass's factor tables for the last eight stages, A[r 8 + sp] for row r and
// stage sp, B[(1 << sp) - 1 + u]; *peak receives the largest magnitude any
// value reached inside the transform.
void fp_forward_ntt(double *x, int logN, double q, const uint64_t *fw, const uint64_t *A, const uint64_t *B,
                    uint64_t *out, double *peak)
{
    const long N = 1l << logN;
    const int LR = logN - 8;
    const double qi = 1.0 / q;
    double pk = 0.0;
    for (long i = 0; i < N; i++) pk = std::fmax(pk, std::fabs(x[i]));
    for (int s = 0; s < logN; s++) {
        const long m = 1l << s, half = N >> (s + 1);
        for (long j = 0; j < m; j++) {
            double w, c;
            if (s < LR) {
                w = (double)fw[m + j];
                c = w / q;
            } else {
                // group j = r 2^sp + u of stage s = LR + sp inside row r
                const int sp = s - LR;
                const long r = j >> sp, u = j & ((1l << sp) - 1);
                const double a = (double)A[r * 8 + sp], b = (double)B[(1l << sp) - 1 + u];
                w = hk::mulm_fp(a, b, b / q, q);
                c = w * qi;
            }
            for (long t = 2 * j * half; t < (2 * j + 1) * half; t++) {
                const double r = hk::mulm_fp(x[t + half], w, c, q);
                const double a = x[t];
                x[t] = a + r;
                x[t + half] = a - r;
                pk = std::fmax(pk, std::fmax(std::fabs(x[t]), std::fabs(x[t + half])));
            }
        }
    }
    for (long i = 0; i < N; i++) out[i] = hk::d2u_mod(x[i], q, qi);
    *peak = pk;
}
}
