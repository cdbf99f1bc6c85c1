// KAN model compiled for encrypted evaluation.
#pragma once
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hekan.h"
#include "ckks.hpp"

namespace hk {

// The inputs [lo, lo + n_in) of a layer that arrive in one ciphertext.
struct Part {
    int lo, n_in;
    long n_blk;              // slots per input block (first layer: n_in S; later: previous d S)
    long width;              // valid slots per block: n_in S
    // n_out x (g+k+1) x n_in: blocks m < g+k hold W_f[o][m][i] = w_s[o][i] c[o][i][m],
    // block g+k holds W_b[o][i] (both linear layers as one product)
    std::vector<double> W;
    // the same weights as two matrices (the paper's two products):
    // n_out x (g+k) x n_in for W_f and n_out x 1 x n_in for W_b
    std::vector<double> Wf, Wb;
    // without lazy combination: W' in row order, n_out x (n_in (g+k)),
    // column i (g+k) + m = w_s[o][i] c[o][i][m]
    std::vector<double> Wrow;
};

struct LayerC {
    int n_in, n_out, g, k;
    long d;       // output period: next power of two >= n_out
    long period;  // the block layout repeats every `period` slots (first layer: N/2)
    std::vector<double> knots, silu;
    double silu_lo, silu_hi;
    std::vector<std::vector<double>> comp;
    double prescale;  // explicit 1/(2R) before PolyComp, 0 = folded
    // first layer: one part per input ciphertext (feature chunks, when the
    // repeat-packed input would not fit the slots); later layers: one part
    std::vector<Part> parts;
};

struct Model {
    Ctx *ctx;
    bool refresh;
    long S;    // input vectors per ciphertext
    int circ;  // HE_CIRCUIT_* restructurings (0: the paper's order)
    bool shared_cmp() const { return (circ & HE_CIRCUIT_SHARED_COMPARISON) != 0; }
    bool fused() const { return (circ & HE_CIRCUIT_FUSED_LINEAR) != 0; }
    bool folded() const { return (circ & HE_CIRCUIT_FOLDED_PERIOD) != 0; }
    bool naive() const { return (circ & HE_CIRCUIT_NAIVE_PERMUTATION) != 0; }
    bool shared_moddown() const { return (circ & HE_CIRCUIT_SHARED_MODDOWN) != 0; }
    std::vector<LayerC> layers;
    std::vector<long> steps;
    std::unordered_map<std::string, Pt> pt_cache;   // Montgomery NTT plaintexts for lincombs
    std::unordered_map<std::string, Buf> add_cache; // NTT plaintexts added to ciphertexts
    Model(Ctx *c, const he_kan_desc *d, bool refresh);
    Model() : ctx(nullptr), refresh(false), S(1), circ(0) {}  // no layers (the evaluators alone)
    size_t n_inputs() const { return layers[0].parts.size(); }
};

// The naive method's permutation of one part's bases: slot (i (g+k) + m) S + s
// receives slot m n_blk + i S + s; off[k] is the signed offset src - dst of
// destination dst[k] (in (-N/4, N/4]), b1 the baby-step width (the power of
// two >= sqrt(2 max|off| + 1)); an offset o = g b1 + b, g = floor(o / b1).
struct PermPlan {
    std::vector<long> dst, off;
    long b1;
};
PermPlan perm_plan(const LayerC &L, const Part &P, long S, long slots);

// in: one ciphertext per part of the layer (the first layer's feature
// chunks, or the previous layer's output)
Ct eval_layer(Ctx &c, Model &m, const Keys &k, const std::vector<Ct> &in, size_t li);
Ct eval_model(Ctx &c, Model &m, const Keys &k, const std::vector<Ct> &in);

// the Chebyshev series cf on [lo, hi] of every slot of x by baby-step
// giant-step (the evaluator of the SiLU approximation)
Ct cheb_series(Ctx &c, const Keys &k, const Ct &x, const std::vector<double> &cf, double lo, double hi);

}  // namespace hk
