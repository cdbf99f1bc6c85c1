// CKKS bootstrapping on the device-resident RNS-CKKS layer.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "ckks.hpp"

namespace hk {

// One group of consecutive butterfly stages of CoeffToSlot (inverse: F_s^H/2
// from the top stage down) or SlotToCoeff (F_s from stage 0 up), as the
// diagonals of its merged matrix without the group's constant.
struct BootGroup {
    std::vector<int> stages;  // application order
    bool inverse;
    long u, b1;               // offsets are multiples of u; baby-step width
    std::map<long, std::pair<std::vector<double>, std::vector<double>>> diag;  // offset -> (re, im)
};

// the group of `stages` (application order); zr, zi: zeta_table of logN
BootGroup boot_group(int logN, const std::vector<int> &stages, bool inverse, const std::vector<double> &zr,
                     const std::vector<double> &zi);

struct Boot {
    Ctx *ctx;
    int cts_levels, stc_levels, r;
    bool real;  // real slot values, SlotToCoeff first (bootstrap_real)
    long slots;  // n: the transforms' period (N/2 unless sparse)
    double K;
    std::vector<double> cf;  // Chebyshev series of cos(2 pi (y - 1/4) / 2^r) on [-K, K]
    std::vector<BootGroup> cts, stc;
    std::vector<long> subsum;  // SubSum's rotation steps n 2^k (sparse only)
    std::vector<long> steps;   // rotation steps, with kStepConjugate
    std::map<std::string, Pt> pt_cache;
    Boot(Ctx *c, int cts_levels, int stc_levels, double K, int r, const std::vector<double> &cf, bool real = false,
         long slots = 0);
};

// refresh of nb ciphertexts (one batch) at a computation level: the result is
// at the top computation level with the same slot values (with b.real: their
// real parts, the input at stc_levels or above)
Ct bootstrap(Ctx &c, Boot &b, const Keys &k, const Ct &in);
// SlotToCoeff scales the slots by this before ModRaise in the real-slot refresh
constexpr double kRealC1 = 1.0 / 128.0;
// its stages: ModRaise and CoeffToSlot of `in`; EvalMod of y; SlotToCoeff of
// the recombined w for an input that was at src_level
Ct boot_coeff_to_slot(Ctx &c, Boot &b, const Keys &k, const Ct &in);
Ct boot_eval_mod(Ctx &c, Boot &b, const Keys &k, const Ct &y);
Ct boot_slot_to_coeff(Ctx &c, Boot &b, const Keys &k, const Ct &w, int src_level);

}  // namespace hk
