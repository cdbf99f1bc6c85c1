// KAN model compiled for encrypted evaluation.
#pragma once
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hekan.h"
#include "ckks.hpp"

namespace hk {

struct LayerC {
    int n_in, n_out, g, k;
    long n_blk;  // slots per input block (first layer: n_in; later: previous d)
    long d;      // output period: next power of two >= n_out
    std::vector<double> knots, silu;
    double silu_lo, silu_hi;
    std::vector<std::vector<double>> comp;
    double prescale;         // explicit 1/(2R) before PolyComp, 0 = folded
    std::vector<double> Wf;  // n_out x (g+k) n_blk, ColTile column order
    std::vector<double> Wb;  // n_out x n_blk
};

struct Model {
    Ctx *ctx;
    bool refresh;
    std::vector<LayerC> layers;
    std::vector<long> steps;
    std::unordered_map<std::string, Pt> pt_cache;   // Montgomery NTT plaintexts for lincombs
    std::unordered_map<std::string, Buf> add_cache; // NTT plaintexts added to ciphertexts
    Model(Ctx *c, const he_kan_desc *d, bool refresh);
};

Ct eval_layer(Ctx &c, Model &m, const Keys &k, const Ct &in, size_t li);
Ct eval_model(Ctx &c, Model &m, const Keys &k, const Ct &in);

}  // namespace hk
