// CKKS bootstrapping: the ciphertext refresh of the paper's Experiment Setup
// (depth 20 with bootstrapping in the settings of Lee et al. 2022, whose
// procedure the paper does not restate), as the full-slot RNS-CKKS
// bootstrapping of Cheon-Han-Kim-Kim-Song 2018, Chen-Chillotti-Song 2019 and
// Han-Ki 2020 on a chain whose top levels use wide primes:
//   ModRaise -> CoeffToSlot (the inverse special DFT of the encoding, its
//   butterfly stages merged into groups, one baby-step giant-step product
//   per group) -> real/imaginary split by conjugation -> EvalMod (Chebyshev
//   series of a scaled cosine, double-angle steps) on both halves in one
//   batch -> recombination -> SlotToCoeff (the special DFT, the last group
//   landing at the top computation level).
// With M = N/2 slots and zeta = exp(i pi / N): U0[j][k] = zeta^(5^j k) =
// F_{m-1} ... F_0 R (R the bit reversal), where F_s maps v to
// out_p = v_p + w v_{p+h} (bit s of p clear) or v_{p-h} - w v_p (set),
// h = 2^s, w = zeta^((5^(p mod h) mod 8h) M / (2h)).  CoeffToSlot multiplies
// by (S_L / (2 q_0)) (F_0^H/2) ... (F_{m-1}^H/2), SlotToCoeff by
// q_0 / (2 pi S_in) F_{m-1} ... F_0, the constant on each one's first group.
// Each merged entry is one path through the butterflies: sign * zeta^e
// (times 2^-stages for F^H/2), its parts the doubles nearest zeta^e's, then
// scaled by the sign and power of two (exact) and the constant (one rounding).
#include "boot.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kan.hpp"

namespace hk {

static long pow2ceil_l(long n)
{
    long p = 1;
    while (p < n) p <<= 1;
    return p;
}
static long floordiv_l(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// stages 0..m-1 in G groups of consecutive stages in application order
// (sizes m / G, the first m % G one larger)
static std::vector<std::vector<int>> stage_groups(int m, int G, bool ascending)
{
    if (G < 1 || G > m) throw HeError(-1, "bootstrapping: stage groups must be between 1 and log2 of the slots");
    std::vector<int> order(m);
    for (int i = 0; i < m; i++) order[i] = ascending ? i : m - 1 - i;
    std::vector<std::vector<int>> out;
    int pos = 0;
    for (int g = 0; g < G; g++) {
        const int n = m / G + (g < m % G ? 1 : 0);
        out.emplace_back(order.begin() + pos, order.begin() + pos + n);
        pos += n;
    }
    return out;
}

BootGroup boot_group(int logN, const std::vector<int> &stages, bool inverse, const std::vector<double> &zr,
                     const std::vector<double> &zi)
{
    const long N = 1l << logN, M = N / 2, twoN = 2 * N;
    BootGroup G;
    G.stages = stages;
    G.inverse = inverse;
    long gmask = 0;
    int smin = 64;
    for (int s : stages) {
        gmask |= 1l << s;
        smin = std::min(smin, s);
    }
    G.u = 1l << smin;
    // twiddle exponents per stage: (5^j mod 8h) M / (2h), j < h
    std::map<int, std::vector<long>> tw;
    for (int s : stages) {
        const long h = 1l << s;
        std::vector<long> e(h);
        long v = 1;
        for (long j = 0; j < h; j++) {
            e[j] = v * (M / (2 * h));
            v = v * 5 % (8 * h);
        }
        tw[s] = e;
    }
    const double f2 = inverse ? std::ldexp(1.0, -(int)stages.size()) : 1.0;
    const int n = (int)stages.size();
    for (long c = 0; c < (1l << n); c++)
        for (long i = 0; i < M; i++) {
            long j = i & ~gmask;
            for (int k = 0; k < n; k++)
                if (c >> k & 1) j |= 1l << stages[k];
            long p = j, e = 0, sg = 1;
            for (int s : stages) {
                const long h = 1l << s;
                const long qi = p;
                p = (p & ~h) | (i & h);
                const int qs = (int)(qi >> s & 1), ps = (int)(p >> s & 1);
                const long w = tw[s][p & (h - 1)];
                if (inverse) {
                    if (ps && qs) sg = -sg;
                    if (ps) e = (e + twoN - w) % twoN;
                } else {
                    if (qs && ps) sg = -sg;
                    if (qs) e = (e + w) % twoN;
                }
            }
            long o = ((j - i) % M + M) % M;
            if (o > M / 2) o -= M;
            auto &d = G.diag[o];
            if (d.first.empty()) {
                d.first.assign(M, 0.0);
                d.second.assign(M, 0.0);
            }
            const double f = (double)sg * f2;
            d.first[i] = f * zr[e];
            d.second[i] = f * zi[e];
        }
    long R = 0;
    for (auto &kv : G.diag) R = std::max(R, std::labs(kv.first));
    R /= G.u;
    long b = 1;
    while (b * b < 2 * R + 1) b++;
    G.b1 = G.u * pow2ceil_l(b);
    return G;
}

Boot::Boot(Ctx *c, int cts, int stc, double K_, int r_, const std::vector<double> &cf_, bool real_, long slots_)
    : ctx(c), cts_levels(cts), stc_levels(stc), r(r_), real(real_), slots(slots_ ? slots_ : c->N / 2), K(K_), cf(cf_)
{
    if (slots < 2 || slots > c->N / 2 || (slots & (slots - 1)))
        throw HeError(-1, "bootstrapping: slots must be a power of two between 2 and N/2");
    int m = 0;
    while ((1l << m) < slots) m++;
    for (long t = slots; t < c->N / 2; t <<= 1) subsum.push_back(t);
    if (!(K > 0.0) || r < 0 || cf.size() < 2) throw HeError(-1, "bootstrapping: bad EvalMod parameters");
    std::vector<double> zr(2l * c->N), zi(2l * c->N);
    zeta_table(c->logN, zr.data(), zi.data());
    for (auto &st : stage_groups(m, cts, false)) this->cts.push_back(boot_group(c->logN, st, true, zr, zi));
    for (auto &st : stage_groups(m, stc, true)) this->stc.push_back(boot_group(c->logN, st, false, zr, zi));
    std::vector<long> s{kStepConjugate};
    s.insert(s.end(), subsum.begin(), subsum.end());
    for (auto *gs : {&this->cts, &this->stc})
        for (const BootGroup &G : *gs)
            for (auto &kv : G.diag) {
                const long g = floordiv_l(kv.first, G.b1), bb = kv.first - g * G.b1;
                if (bb) s.push_back(bb);
                if (g) s.push_back(g * G.b1);
            }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    steps = s;
}

// sum_o diag_o * rot(x, o) times cst at level t by baby-step giant-step:
// sum_g rot( sum_b rot(diag_(g b1 + b), -g b1) * rot(x, b), g b1 ); the
// baby rotations share one ModUp, the giant rotations one ModDown
static Ct lintrans(Ctx &c, Boot &bt, const Keys &k, const BootGroup &G, const std::string &tag, double cst,
                   const Ct &x, int t)
{
    const long M = c.N / 2;
    std::map<long, std::vector<long>> giants;  // giant -> babies present
    std::vector<long> babies;
    for (auto &kv : G.diag) {
        const long g = floordiv_l(kv.first, G.b1);
        giants[g].push_back(kv.first - g * G.b1);
        babies.push_back(kv.first - g * G.b1);
    }
    std::sort(babies.begin(), babies.end());
    babies.erase(std::unique(babies.begin(), babies.end()), babies.end());
    Ct xd = c.mod_drop(x, t + 1);
    u64 cb;
    std::memcpy(&cb, &cst, 8);
    auto key = [&](long g, long b) {
        return tag + "g" + std::to_string(g) + "b" + std::to_string(b) + "|" + std::to_string(t) + "|" +
               std::to_string(xd.level) + "|" + std::to_string(cb);
    };
    // the plaintexts not cached yet, encoded together (host encodings in parallel)
    {
        std::vector<std::string> keys;
        std::vector<std::vector<double>> res, ims;
        for (auto &gg : giants)
            for (long b : gg.second) {
                const std::string kk = key(gg.first, b);
                if (bt.pt_cache.count(kk)) continue;
                const auto &d = G.diag.at(gg.first * G.b1 + b);
                const long sh = gg.first * G.b1;
                std::vector<double> re(M), im(M);
                for (long j = 0; j < M; j++) {
                    const long src = ((j - sh) % M + M) % M;
                    re[j] = d.first[src] * cst;
                    im[j] = d.second[src] * cst;
                }
                keys.push_back(kk);
                res.push_back(std::move(re));
                ims.push_back(std::move(im));
            }
        if (!keys.empty()) {
            std::vector<const std::vector<double> *> zr, zi;
            for (size_t i = 0; i < keys.size(); i++) {
                zr.push_back(&res[i]);
                zi.push_back(&ims[i]);
            }
            const double X = c.S[t] * (double)c.q[t + 1] / c.S[xd.level];
            std::vector<Pt> pts = c.vec_pts(zr, X, t + 2, &zi);
            for (size_t i = 0; i < keys.size(); i++) bt.pt_cache.emplace(keys[i], pts[i]);
        }
    }
    std::vector<Ct> rots = c.rotate_many(xd, babies, k);
    std::vector<Ct> inner;
    inner.reserve(giants.size());
    std::vector<std::pair<const Ct *, long>> items;
    for (auto &gg : giants) {
        std::vector<std::pair<const Ct *, const Pt *>> terms;
        for (long b : gg.second) {
            const size_t bi = std::lower_bound(babies.begin(), babies.end(), b) - babies.begin();
            terms.push_back({&rots[bi], &bt.pt_cache.at(key(gg.first, b))});
        }
        inner.push_back(c.lincomb(terms, t));
        items.push_back({&inner.back(), gg.first * G.b1});
    }
    return c.rotate_sum(items, k);
}

// two batches of one level as one: [l+1][nb_a + nb_b][2][N]
static Ct concat(Ctx &c, const Ct &a, const Ct &b)
{
    Ct o = c.new_ct(a.level, a.nb + b.nb);
    const long ls = 2l * c.N * o.nb;
    launch_copy(PolySet{o.d(), ls, (long)c.N, a.level + 1, 2 * a.nb}, c.ctset(a), c.N, c.st);
    launch_copy(PolySet{o.d() + 2l * c.N * a.nb, ls, (long)c.N, b.level + 1, 2 * b.nb}, c.ctset(b), c.N, c.st);
    c.n_launch += 2;
    return o;
}

// elements [e0, e0 + n) of a batch
static Ct slice(Ctx &c, const Ct &a, int e0, int n)
{
    Ct o = c.new_ct(a.level, n);
    launch_copy(c.ctset(o), PolySet{a.d() + 2l * c.N * e0, 2l * c.N * a.nb, (long)c.N, a.level + 1, 2 * n}, c.N,
                c.st);
    c.n_launch++;
    return o;
}

Ct boot_coeff_to_slot(Ctx &c, Boot &b, const Keys &k, const Ct &in)
{
    if (in.level < 0 || in.level > c.top) throw HeError(-1, "bootstrapping: the input must be at a computation level");
    const double q0 = (double)c.q[0];
    Ct x = c.mod_raise(c.mod_drop(in, 0));
    // sparse: SubSum makes the slots n-periodic (times N/(2n), undone by the
    // first group's constant)
    for (long t : b.subsum) x = c.rotate_add(x, t, x, k);
    const double sub = (double)b.slots / (double)(c.N / 2);
    for (size_t gi = 0; gi < b.cts.size(); gi++) {
        if (x.level < 1) throw HeError(-3, "bootstrapping does not fit the levels");
        const double cst = gi == 0 ? c.S[c.L] / (2.0 * q0) * sub : 1.0;
        x = lintrans(c, b, k, b.cts[gi], "C" + std::to_string(gi), cst, x, x.level - 1);
    }
    return x;
}

Ct boot_eval_mod(Ctx &c, Boot &b, const Keys &k, const Ct &y)
{
    Ct u = cheb_series(c, k, y, b.cf, -b.K, b.K);
    const double m1 = -1.0;
    for (int i = 0; i < b.r; i++) {
        if (u.level < 1) throw HeError(-3, "bootstrapping does not fit the levels");
        u = c.mul_affine(u, u, k, 2, &m1);
    }
    return u;
}

Ct boot_slot_to_coeff(Ctx &c, Boot &b, const Keys &k, const Ct &w_in, int src_level)
{
    if (src_level < 0 || src_level > c.top) throw HeError(-1, "bootstrapping: bad source level");
    const double q0 = (double)c.q[0];
    Ct w = w_in;
    for (size_t gi = 0; gi < b.stc.size(); gi++) {
        const bool last = gi + 1 == b.stc.size();
        const int t = last ? c.top : w.level - 1;
        if (t < c.top || t >= w.level) throw HeError(-3, "bootstrapping does not fit the levels");
        const double cst = gi == 0 ? q0 / (2.0 * M_PI * c.S[src_level]) : 1.0;
        w = lintrans(c, b, k, b.stc[gi], "S" + std::to_string(gi), cst, w, t);
    }
    return w;
}

// Real slot values with SlotToCoeff first (Chen-Chillotti-Song 2019): the
// special DFT F_{m-1} ... F_0 times kRealC1 runs on the input's own limbs, so
// the plaintext's low coefficients become S kRealC1 R z (S the scale there);
// after ModRaise and CoeffToSlot, w + conj(w) = S kRealC1 z / q_0 + integers
// in natural slot order, one EvalMod gives 2 pi S kRealC1 z / q_0 (the
// imaginary half holds no message and is dropped), and one product by
// q_0 / (2 pi S kRealC1) lands at the top computation level.
static Ct bootstrap_real(Ctx &c, Boot &b, const Keys &k, const Ct &in)
{
    if (in.level > c.top || in.level < (int)b.stc.size())
        throw HeError(-1, "real-slot bootstrapping: the input must be at a computation level of at least stc_levels");
    Ct x = in;
    for (size_t gi = 0; gi < b.stc.size(); gi++)
        x = lintrans(c, b, k, b.stc[gi], "F" + std::to_string(gi), gi == 0 ? kRealC1 : 1.0, x, x.level - 1);
    const int lp = x.level;
    Ct w = boot_coeff_to_slot(c, b, k, x);
    Ct u = boot_eval_mod(c, b, k, c.add(w, c.rotate(w, kStepConjugate, k)));
    if (u.level <= c.top) throw HeError(-3, "bootstrapping does not fit the levels");
    const double kinv = (double)c.q[0] / (2.0 * M_PI * c.S[lp] * kRealC1);
    Pt p = c.const_pt(kinv, c.S[c.top] * (double)c.q[c.top + 1] / c.S[u.level], c.top + 2);
    return c.lincomb({{&u, &p}}, c.top);
}

Ct bootstrap(Ctx &c, Boot &b, const Keys &k, const Ct &in)
{
    if (b.real) return bootstrap_real(c, b, k, in);
    Ct x = boot_coeff_to_slot(c, b, k, in);
    Ct xc = c.rotate(x, kStepConjugate, k);
    // both halves through EvalMod in one batch
    Ct u = boot_eval_mod(c, b, k, concat(c, c.add(x, xc), c.mul_i(c.sub(xc, x))));
    Ct w = c.add(slice(c, u, 0, in.nb), c.mul_i(slice(c, u, in.nb, in.nb)));
    return boot_slot_to_coeff(c, b, k, w, in.level);
}

}  // namespace hk
