// Encrypted KAN evaluation on the device-resident RNS-CKKS layer (Method):
//   * SiLU Approximation: Chebyshev series by baby-step giant-step;
//   * B-spline Basis Approximation: Fast Repeat Packing (Algorithm 1) and the
//     comparison-based order-0 bases with the order-k recursion (Algorithm 2);
//   * Lazy Combination and Fusion Linear Layer: W' = W_s o C permuted by the
//     Algorithm 3 permutation into W_f, applied with the hybrid diagonal
//     method and baby-step giant-step rotations.
// The placement of every rescale and the scale of every plaintext is fixed so
// that all ciphertexts at level l carry the canonical scale S_l.
#include "kan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace hk {

static int clog2i(long n)
{
    int r = 0;
    while ((1l << r) < n) r++;
    return r;
}
static long pow2ceil(long n) { return 1l << clog2i(n); }
static long floordiv(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

PermPlan perm_plan(const LayerC &L, const Part &P, long S, long slots)
{
    const long nb = L.g + L.k;
    PermPlan pp;
    long R = 0;
    for (long i = 0; i < P.n_in; i++)
        for (long m = 0; m < nb; m++)
            for (long s = 0; s < S; s++) {
                const long d = (i * nb + m) * S + s;
                long o = ((m * P.n_blk + i * S + s - d) % slots + slots) % slots;
                if (o > slots / 2) o -= slots;
                pp.dst.push_back(d);
                pp.off.push_back(o);
                R = std::max(R, std::labs(o));
            }
    long b = 1;
    while (b * b < 2 * R + 1) b++;
    pp.b1 = pow2ceil(b);
    return pp;
}

// ------------------------------------------------------------------- model
Model::Model(Ctx *c, const he_kan_desc *d, bool refresh_) : ctx(c), refresh(refresh_)
{
    if (!d || d->n_layers < 1 || !d->layers) throw HeError(-1, "model: empty description");
    const long slots = ctx->N / 2;
    S = d->samples_per_ct <= 0 ? 1 : d->samples_per_ct;
    if ((S & (S - 1)) != 0 || S > slots) throw HeError(-1, "model: samples per ciphertext must be a power of two");
    circ = d->circuit;
    if (circ & ~(HE_CIRCUIT_RESTRUCTURED | HE_CIRCUIT_NAIVE_PERMUTATION))
        throw HeError(-1, "model: unknown circuit option");
    if (naive() && (fused() || folded()))
        throw HeError(-1, "model: the naive permutation excludes the fused linear layers and the folded period");
    long n_blk = 0;
    for (int li = 0; li < d->n_layers; li++) {
        const he_kan_layer &s = d->layers[li];
        if (s.n_in < 1 || s.n_out < 1 || s.g < 1 || s.k < 0) throw HeError(-1, "model: bad layer shape");
        if (li > 0 && (long)s.n_in * S > n_blk) throw HeError(-1, "model: layer widths do not chain");
        if (!s.knots || !s.wb || !s.ws || !s.c || !s.silu_coeffs || s.silu_degree < 1 || s.comp_stages < 1 ||
            !s.comp_stage_len || !s.comp_coeffs || !(s.silu_hi > s.silu_lo))
            throw HeError(-1, "model: missing layer data");
        LayerC L;
        L.n_in = s.n_in;
        L.n_out = s.n_out;
        L.g = s.g;
        L.k = s.k;
        L.d = pow2ceil(s.n_out);
        const int r = s.g + 2 * s.k + 1, nb = s.g + s.k;
        L.knots.assign(s.knots, s.knots + r);
        L.silu.assign(s.silu_coeffs, s.silu_coeffs + s.silu_degree + 1);
        L.silu_lo = s.silu_lo;
        L.silu_hi = s.silu_hi;
        L.prescale = s.comp_prescale;
        int off = 0;
        for (int st = 0; st < s.comp_stages; st++) {
            int len = s.comp_stage_len[st];
            if (len < 2 || len > 4) throw HeError(-1, "model: comparison stage must have degree 3, 5 or 7");
            L.comp.emplace_back(s.comp_coeffs + off, s.comp_coeffs + off + len);
            off += len;
        }
        if (L.d * S > slots) throw HeError(-4, "model: n_out S exceeds N/2 slots");
        // packing: the first layer makes 2^ceil(log2(g+2k)) copies of its input
        // (Algorithm 1); when n_in S copies do not fit the slots the input comes
        // as feature chunks, each as wide as the copies allow (cap =
        // slots / 2^ceil(log2(g+2k)) / S features), the last one the rest;
        // later layers need (g+2k) blocks of the previous output period
        long cap = s.n_in;
        if (li == 0) {
            cap = slots / pow2ceil(r - 1) / S;
            if (cap < 1) throw HeError(-4, "model: g+2k copies of one input exceed N/2 slots");
        } else if ((long)(r - 1) * n_blk > slots) {
            throw HeError(-4, "model: n_in (g+2k) exceeds N/2 slots");
        }
        for (long lo = 0; lo < s.n_in; lo += cap) {
            Part P;
            P.lo = (int)lo;
            P.n_in = (int)std::min(cap, (long)s.n_in - lo);
            P.width = (long)P.n_in * S;
            P.n_blk = li == 0 ? P.width : n_blk;
            // fused weights W_f[o][m][i] = w_s[o][i] c[o][i][m] (W' P with the
            // Algorithm 3 permutation: column j_c = m n_i + i of W_f is column
            // j_r = i (g+k) + m of W'), then W_b[o][i] as block g+k, over the
            // part's inputs; their slot layout (block m at m n_blk, input i of
            // vector v at i S + v) is formed when the diagonals are
            P.W.assign((size_t)s.n_out * (nb + 1) * P.n_in, 0.0);
            P.Wf.assign((size_t)s.n_out * nb * P.n_in, 0.0);
            P.Wb.assign((size_t)s.n_out * P.n_in, 0.0);
            for (int o = 0; o < s.n_out; o++)
                for (int i = 0; i < P.n_in; i++) {
                    const size_t e = (size_t)o * s.n_in + P.lo + i;
                    const double ws = s.ws[e];
                    for (int m = 0; m < nb; m++) {
                        P.W[((size_t)o * (nb + 1) + m) * P.n_in + i] = ws * s.c[e * nb + m];
                        P.Wf[((size_t)o * nb + m) * P.n_in + i] = ws * s.c[e * nb + m];
                    }
                    P.W[((size_t)o * (nb + 1) + nb) * P.n_in + i] = s.wb[e];
                    P.Wb[(size_t)o * P.n_in + i] = s.wb[e];
                }
            if (naive()) {
                P.Wrow.assign((size_t)s.n_out * P.n_in * nb, 0.0);
                for (int o = 0; o < s.n_out; o++)
                    for (int i = 0; i < P.n_in; i++)
                        for (int m = 0; m < nb; m++)
                            P.Wrow[((size_t)o * P.n_in + i) * nb + m] = s.ws[(size_t)o * s.n_in + P.lo + i] *
                                                                        s.c[((size_t)o * s.n_in + P.lo + i) * nb + m];
            }
            L.parts.push_back(std::move(P));
        }
        // a hidden layer's input repeats every n_blk slots, so its whole block
        // layout (g+2k comparison blocks, g+2k+1 when the second comparison is
        // shared or the masked SiLU needs block g of a k = 0 layer) can repeat
        // every next power of two of that many slots; the products then repeat
        // likewise and the fold runs over one period.  Otherwise the layout
        // spans all slots.
        const long nblocks = (shared_cmp() || (fused() && s.k == 0)) ? r : r - 1;
        L.period = (li == 0 || !folded()) ? slots : std::min(slots, pow2ceil(nblocks * n_blk));
        layers.push_back(std::move(L));
        n_blk = layers.back().d * S;
    }
    // rotation steps
    std::vector<long> st;
    for (size_t li = 0; li < layers.size(); li++) {
        const LayerC &L = layers[li];
        for (const Part &P : L.parts) {
            if (li == 0)
                for (int j = 1; j <= clog2i(L.g + 2 * L.k); j++) st.push_back(-P.n_blk * (1l << (j - 1)));
            st.push_back(P.n_blk);
            if (naive()) {
                const PermPlan pp = perm_plan(L, P, S, slots);
                for (long o : pp.off) {
                    const long g = floordiv(o, pp.b1), b = o - g * pp.b1;
                    if (b) st.push_back(b);
                    if (g) st.push_back(g * pp.b1);
                }
            }
        }
        const long D = L.d * S;
        int b1 = 1 << ((clog2i(L.d) + 1) / 2);
        long g1 = L.d / b1;
        for (int b = 1; b < b1; b++) st.push_back(b * S);
        for (long gi = 1; gi < g1; gi++) st.push_back(gi * b1 * S);
        for (long s = L.period / 2; s >= D; s /= 2) st.push_back(s);
    }
    std::sort(st.begin(), st.end());
    st.erase(std::unique(st.begin(), st.end()), st.end());
    steps = st;
}

// ------------------------------------------------------------- evaluator
struct Eval {
    Ctx &c;
    const Keys &k;
    Model &m;
    Eval(Ctx &c_, const Keys &k_, Model &m_) : c(c_), k(k_), m(m_) {}

    double X(int t, int lct) const
    {
        if (t < 0) throw HeError(-3, "the circuit needs more levels than its input has");
        return c.S[t] * (double)c.q[t + 1] / c.S[lct];
    }

    // sum_i c_i x_i at level t [+ *cst]
    Ct lin_scalar(const std::vector<std::pair<const Ct *, double>> &terms, int t, const double *cst = nullptr)
    {
        std::vector<Pt> pts;
        pts.reserve(terms.size());
        for (auto &tm : terms) pts.push_back(c.const_pt(tm.second, X(t, tm.first->level), t + 2));
        std::vector<std::pair<const Ct *, const Pt *>> v;
        for (size_t i = 0; i < terms.size(); i++) v.push_back({terms[i].first, &pts[i]});
        return c.lincomb(v, t, cst);
    }

    // cached slot-vector plaintext for a lincomb term: key + target + operand level
    const Pt &vec(const std::string &key, int t, int lct, const std::vector<double> &z)
    {
        std::string full = key + "|" + std::to_string(t) + "|" + std::to_string(lct);
        auto it = m.pt_cache.find(full);
        if (it != m.pt_cache.end()) return it->second;
        Pt p = c.vec_pt(z.data(), z.size(), X(t, lct), t + 2);
        return m.pt_cache.emplace(full, p).first->second;
    }

    const Buf &addvec(const std::string &key, int level, const std::vector<double> &z)
    {
        std::string full = key + "|a|" + std::to_string(level);
        auto it = m.add_cache.find(full);
        if (it != m.add_cache.end()) return it->second;
        Buf b = c.encode_ntt(z.data(), z.size(), c.S[level], level + 1, false);
        return m.add_cache.emplace(full, b).first->second;
    }

    Ct mul(const Ct &a, const Ct &b) { return c.mul(a, b, k); }
    // km (a b) [+ cc], the factor and constant applied in the rescale
    Ct mul_aff(const Ct &a, const Ct &b, long km, const double *cc) { return c.mul_affine(a, b, k, km, cc); }

    // sum_i a_i v^(2i+1) [+ *cst], degree 3 / 5 / 7 in depth 2 / 3 / 3
    Ct odd_poly(const Ct &v, const std::vector<double> &a, const double *cst = nullptr)
    {
        const int l = v.level;
        if (a.size() == 2) {
            Ct v2 = mul(v, v);
            Ct t3 = mul(lin_scalar({{&v, a[1]}}, l - 1), v2);
            return c.add(lin_scalar({{&v, a[0]}}, l - 2, cst), t3);
        }
        if (a.size() == 3) {
            Ct v2 = mul(v, v);
            Ct v4 = mul(v2, v2);
            Ct t3 = mul(lin_scalar({{&v, a[1]}}, l - 1), v2);
            Ct t5 = mul(lin_scalar({{&v, a[2]}}, l - 2), v4);
            return c.add(lin_scalar({{&v, a[0]}, {&t3, 1.0}}, l - 3, cst), t5);
        }
        Ct v2 = mul(v, v);
        Ct v4 = mul(v2, v2);
        Ct t3 = mul(lin_scalar({{&v, a[1]}}, l - 1), v2);
        Ct t7 = mul(lin_scalar({{&v, a[3]}}, l - 1), v2);
        Ct B = c.add(t7, lin_scalar({{&v, a[2]}}, l - 2));
        Ct Cc = mul(B, v4);
        return c.add(lin_scalar({{&v, a[0]}, {&t3, 1.0}}, l - 3, cst), Cc);
    }

    // the composite plus 1/2 (the constant joins the last stage's rescale)
    Ct polycomp(Ct v, const std::vector<std::vector<double>> &stages)
    {
        const double half = 0.5;
        if (stages.empty()) return c.add_const(v, half);
        for (size_t i = 0; i < stages.size(); i++) v = odd_poly(v, stages[i], i + 1 == stages.size() ? &half : nullptr);
        return v;
    }

    // ---- Chebyshev series by baby-step giant-step
    struct Cheb {
        Eval &e;
        std::map<long, Ct> T;
        long b;
        const std::vector<double> *mask = nullptr;  // every coefficient times this slot vector
        std::string tag;                            // plaintext cache key prefix (masked leaves)
        Cheb(Eval &e_) : e(e_) {}
        std::vector<double> masked(double v) const
        {
            std::vector<double> z(*mask);
            for (auto &x : z) x *= v;
            return z;
        }
        // sum_i T_i cf_i (i in 1..n-1) at level t, plus cf_0 when with_const;
        // `path` names the leaf for the plaintext cache
        Ct leaf(const std::vector<std::pair<const Ct *, double>> &terms, double c0, bool with_const, int t,
                const std::string &path)
        {
            if (!mask) {
                return e.lin_scalar(terms, t, with_const ? &c0 : nullptr);
            }
            std::vector<std::pair<const Ct *, const Pt *>> v;
            for (size_t i = 0; i < terms.size(); i++)
                v.push_back({terms[i].first,
                             &e.vec(tag + path + "/" + std::to_string(i), t, terms[i].first->level,
                                    masked(terms[i].second))});
            Ct s = e.c.lincomb(v, t);
            return with_const ? e.c.add_plain(s, e.addvec(tag + path + "/c", t, masked(c0))) : s;
        }
        long giant(long n) const
        {
            long G = b;
            while (2 * G < n) G *= 2;
            return G;
        }
        static void split(const std::vector<double> &cf, long G, std::vector<double> &q, std::vector<double> &r)
        {
            long n = (long)cf.size();
            q.assign(n - G, 0.0);
            q[0] = cf[G];
            for (long j = 1; j < n - G; j++) q[j] = 2.0 * cf[G + j];
            r.assign(cf.begin(), cf.begin() + G);
            for (long j = 1; j < n - G; j++) r[G - j] = r[G - j] - cf[G + j];
        }
        bool feasible(const std::vector<double> &cf, int t)
        {
            long n = (long)cf.size();
            if (n <= b) {
                int mn = 1 << 30;
                for (long i = 1; i < n; i++) mn = std::min(mn, T.at(i).level);
                return t <= mn - 1;
            }
            long G = giant(n);
            std::vector<double> q, r;
            split(cf, G, q, r);
            bool okq = q.size() == 1 ? t <= T.at(G).level - 1 : (t + 1 <= T.at(G).level && feasible(q, t + 1));
            return okq && feasible(r, t);
        }
        Ct rec(const std::vector<double> &cf, int t, const std::string &path = "")
        {
            long n = (long)cf.size();
            if (n <= b) {
                std::vector<std::pair<const Ct *, double>> terms;
                for (long i = 1; i < n; i++) terms.push_back({&T.at(i), cf[i]});
                return leaf(terms, cf[0], true, t, path);
            }
            long G = giant(n);
            std::vector<double> q, r;
            split(cf, G, q, r);
            Ct prod;
            if (q.size() == 1) {
                prod = leaf({{&T.at(G), q[0]}}, 0.0, false, t, path + "g");
            } else {
                Ct qc = rec(q, t + 1, path + "q");
                prod = e.mul(qc, e.c.level_down(T.at(G), t + 1));
            }
            return e.c.add(prod, rec(r, t, path + "r"));
        }
    };

    // the series on every slot of x; with a mask every coefficient (and so the
    // result) is multiplied slot-wise by it, at no extra depth
    Ct cheb_eval(const Ct &x, const std::vector<double> &cf, double lo, double hi,
                 const std::vector<double> *mask = nullptr, const std::string &tag = "")
    {
        Cheb ch(*this);
        ch.mask = mask;
        ch.tag = tag;
        const long deg = (long)cf.size() - 1;
        const int mm = clog2i(deg + 1);
        ch.b = 1l << ((mm + 1) / 2);
        const double alpha = 2.0 / (hi - lo), beta = -(hi + lo) / (hi - lo);
        ch.T[1] = lin_scalar({{&x, alpha}}, x.level - 1, &beta);
        for (long i = 2; i <= ch.b; i++) {
            if (i % 2 == 0) {
                const Ct &h = ch.T.at(i / 2);
                const double m1 = -1.0;
                ch.T[i] = mul_aff(h, h, 2, &m1);
            } else {
                const Ct &a = ch.T.at((i - 1) / 2), &b2 = ch.T.at((i + 1) / 2);
                int lv = std::min(a.level, b2.level);
                Ct p = mul_aff(c.level_down(a, lv), c.level_down(b2, lv), 2, nullptr);
                ch.T[i] = c.sub(p, c.level_down(ch.T.at(1), p.level));
            }
        }
        for (long G = 2 * ch.b; G < deg + 1; G *= 2) {
            const Ct &h = ch.T.at(G / 2);
            const double m1 = -1.0;
            ch.T[G] = mul_aff(h, h, 2, &m1);
        }
        int t = ch.T.at(1).level - 1;
        while (!ch.feasible(cf, t)) {
            t--;
            if (t < 0) throw HeError(-3, "Chebyshev series does not fit the level budget");
        }
        return ch.rec(cf, t);
    }

    // ---- packing and bases
    Ct repeat_pack(Ct x, long n_blk, int nlog)
    {
        for (int j = 1; j <= nlog; j++) x = c.rotate_add(x, -n_blk * (1l << (j - 1)), x, k);
        return x;
    }

    // copy the first `period` entries of v over the rest of it
    static void tile(std::vector<double> &v, long period)
    {
        for (size_t j = (size_t)period; j < v.size(); j++) v[j] = v[j - period];
    }

    // ColTile(G, lo, hi): block mb (< hi-lo) holds t_{lo+mb} for the part's
    // inputs, the layout repeated every L.period slots
    std::vector<double> coltile(const LayerC &L, const Part &P, int lo, int hi) const
    {
        std::vector<double> v(c.N / 2, 0.0);
        for (int mb = 0; mb < hi - lo; mb++)
            for (long i = 0; i < P.width; i++) v[(size_t)mb * P.n_blk + i] = L.knots[lo + mb - 1];
        tile(v, L.period);
        return v;
    }

    // Algorithm 2 on the repeat-packed xr.  shared: xr holds the input in
    // g+2k+1 blocks and the second comparison is taken from the first: the
    // composite is odd, so S((t_{m+2} - x)/2R) = 1 - S((x - t_{m+2})/2R), which
    // is 1 minus the first comparison of block m+1 (one rotation instead of a
    // second PolyComp)
    Ct bspline(const Ct &xr, const LayerC &L, const Part &P, const std::string &tag, bool shared)
    {
        const int r = L.g + 2 * L.k + 1;
        Ct x1, x2;
        if (shared) {
            std::vector<double> g1 = coltile(L, P, 1, r + 1);
            if (L.prescale != 0.0) {
                const double sc = L.prescale;
                for (auto &v : g1) v = -(v * sc);
                const int l1 = xr.level - 1;
                x1 = polycomp(c.add_plain(lin_scalar({{&xr, sc}}, l1), addvec(tag + "g1s", l1, g1)), L.comp);
            } else {
                for (auto &v : g1) v = -v;
                x1 = polycomp(c.add_plain(xr, addvec(tag + "g1", xr.level, g1)), L.comp);
            }
            const double one = 1.0;
            x2 = c.affine(c.rotate(x1, P.n_blk, k), -1, &one, nullptr);
            return bases(mul(x1, x2), xr, L, P, tag);
        }
        std::vector<double> g1 = coltile(L, P, 1, r), g2 = coltile(L, P, 2, r + 1);
        if (L.prescale != 0.0) {
            // (x - g1) / 2R and (g2 - x) / 2R, one rescale each (Algorithm 2)
            const double sc = L.prescale;
            for (auto &v : g1) v = -(v * sc);
            for (auto &v : g2) v = v * sc;
            const int l1 = xr.level - 1;
            x1 = polycomp(c.add_plain(lin_scalar({{&xr, sc}}, l1), addvec(tag + "g1s", l1, g1)), L.comp);
            x2 = polycomp(c.add_plain(lin_scalar({{&xr, -sc}}, l1), addvec(tag + "g2s", l1, g2)), L.comp);
        } else {
            for (auto &v : g1) v = -v;
            x1 = polycomp(c.add_plain(xr, addvec(tag + "g1", xr.level, g1)), L.comp);
            x2 = polycomp(c.affine(xr, -1, nullptr, &addvec(tag + "g2", xr.level, g2)), L.comp);
        }
        return bases(mul(x1, x2), xr, L, P, tag);
    }

    // the k recursion rounds of Algorithm 2 from the order-0 bases b
    Ct bases(Ct b, const Ct &xr, const LayerC &L, const Part &P, const std::string &tag)
    {
        const int r = L.g + 2 * L.k + 1;
        const size_t S2 = c.N / 2;
        for (int j = 1; j <= L.k; j++) {
            const int nbl = r - j - 1;
            std::vector<double> t1 = coltile(L, P, 1, r - j), t2 = coltile(L, P, j + 1, r);
            std::vector<double> t3 = coltile(L, P, j + 2, r + 1), t4 = coltile(L, P, 2, r - j + 1);
            std::vector<double> A1(S2, 0.0), A2n(S2, 0.0), c1(S2, 0.0), c2(S2, 0.0);
            for (int mb = 0; mb < nbl; mb++)
                for (long i = 0; i < P.width; i++) {
                    size_t s = (size_t)mb * P.n_blk + i;
                    double a1 = 1.0 / (t2[s] - t1[s]);
                    double a2 = 1.0 / (t3[s] - t4[s]);
                    A1[s] = a1;
                    A2n[s] = -a2;
                    c1[s] = -(t1[s] * a1);
                    c2[s] = t3[s] * a2;
                }
            tile(A1, L.period);
            tile(A2n, L.period);
            tile(c1, L.period);
            tile(c2, L.period);
            const int lb = b.level;
            std::string jt = tag + "r" + std::to_string(j);
            const Pt &pA1 = vec(jt + "A1", lb, xr.level, A1);
            const Pt &pA2 = vec(jt + "A2", lb, xr.level, A2n);
            Ct P1 = c.add_plain(c.lincomb({{&xr, &pA1}}, lb), addvec(jt + "c1", lb, c1));
            Ct P2 = c.add_plain(c.lincomb({{&xr, &pA2}}, lb), addvec(jt + "c2", lb, c2));
            Ct rb = c.rotate(b, P.n_blk, k);
            Tensor tt = c.tensor(P1, b);
            c.tensor_acc(tt, P2, rb);
            b = c.relin_rescale(tt, k);
        }
        return b;
    }

    // Weights of one linear layer in the slot layout: output o of vector v in
    // row o S + v; column m n_blk + i S + v holds input i of vector v in
    // block m (W (x) I_S over nblocks blocks of n_in inputs).  W is
    // [rows][nblocks][n_in].
    struct SlotMatrix {
        const std::vector<double> &W;
        long n_out, nblocks, n_in, n_blk, S;
        double at(long r, long col) const
        {
            const long o = r / S, v = r % S, mb = col / n_blk, rem = col % n_blk, i = rem / S;
            if (o >= n_out || mb >= nblocks || i >= n_in || rem % S != v) return 0.0;
            return W[((size_t)o * nblocks + mb) * n_in + i];
        }
    };

    // generalised diagonal i of M for output period D and an input repeating
    // every `period` slots, pre-rotated by sh (np.roll): entry j is
    // M[j mod D][(j + i) mod period]
    static std::vector<double> diag(const SlotMatrix &M, long D, long i, long sh, long slots, long period)
    {
        std::vector<double> v(slots, 0.0);
        for (long j = 0; j < slots; j++) {
            long jj = ((j - sh) % slots + slots) % slots;
            v[j] = M.at(jj % D, (jj + i) % period);
        }
        return v;
    }

    // z = sum_{i<d} diag_{iS} * rot(x, iS) by baby-step giant-step at level t;
    // with S vectors per ciphertext only the multiples of S are non-zero
    // diagonals of W (x) I_S, so the d terms use rotations by multiples of S
    Ct matvec(const Ct &x, const SlotMatrix &M, long d, int t, long period, const std::string &tag)
    {
        const long slots = c.N / 2, S = m.S, D = d * S;
        const int b1 = 1 << ((clog2i(d) + 1) / 2);
        const long g1 = d / b1;
        Ct xd = c.mod_drop(x, t + 1);
        // baby steps share one ModUp (hoisting; same residues as separate rotations)
        std::vector<long> bsteps;
        for (int bi = 0; bi < b1; bi++) bsteps.push_back(bi * S);
        std::vector<Ct> rots = c.rotate_many(xd, bsteps, k);
        Ct z;
        bool have = false;
        // with the shared ModDown: the giant steps' inner sums, rotated and
        // summed by one rotate_sum
        std::vector<Ct> inner_g;
        inner_g.reserve(g1);
        std::vector<std::pair<const Ct *, long>> items;
        for (long gi = 0; gi < g1; gi++) {
            std::vector<std::pair<const Ct *, const Pt *>> terms;
            for (int bi = 0; bi < b1; bi++) {
                std::string key = tag + "d" + std::to_string(gi) + "_" + std::to_string(bi);
                std::string full = key + "|" + std::to_string(t) + "|" + std::to_string(xd.level);
                const Pt *pp;
                auto it = m.pt_cache.find(full);
                if (it != m.pt_cache.end()) {
                    pp = &it->second;
                } else {
                    std::vector<double> dv = diag(M, D, (gi * b1 + bi) * S, gi * b1 * S, slots, period);
                    pp = &vec(key, t, xd.level, dv);
                }
                terms.push_back({&rots[bi], pp});
            }
            Ct inner = c.lincomb(terms, t);
            if (m.shared_moddown()) {
                inner_g.push_back(inner);
                items.push_back({&inner_g.back(), gi * b1 * S});
                continue;
            }
            if (!have) {
                z = gi ? c.rotate(inner, gi * b1 * S, k) : inner;
                have = true;
            } else {
                z = gi ? c.rotate_add(inner, gi * b1 * S, z, k) : c.add(z, inner);
            }
        }
        return m.shared_moddown() ? c.rotate_sum(items, k) : z;
    }

    // the naive method's permutation of the bases b into row order at level t
    // (zeros outside the n_in (g+k) S destinations): diagonal method with
    // baby-step giant-step rotations, one plaintext per distinct offset,
    // z = sum_g rot(sum_b rot(diag_(g b1 + b), -g b1) * rot(b, b), g b1)
    Ct permute(const Ct &x, const LayerC &L, const Part &P, int t, const std::string &tag)
    {
        const long slots = c.N / 2;
        const PermPlan pp = perm_plan(L, P, m.S, slots);
        std::map<long, std::map<long, std::vector<long>>> groups;  // giant -> baby -> destinations
        for (size_t k2 = 0; k2 < pp.off.size(); k2++) {
            const long g = floordiv(pp.off[k2], pp.b1);
            groups[g][pp.off[k2] - g * pp.b1].push_back(pp.dst[k2]);
        }
        std::vector<long> babies;
        for (auto &gg : groups)
            for (auto &bb : gg.second) babies.push_back(bb.first);
        std::sort(babies.begin(), babies.end());
        babies.erase(std::unique(babies.begin(), babies.end()), babies.end());
        Ct xd = c.mod_drop(x, t + 1);
        auto full_key = [&](long g, long b) {
            return tag + "g" + std::to_string(g) + "b" + std::to_string(b) + "|" + std::to_string(t) + "|" +
                   std::to_string(xd.level);
        };
        // the diagonals not cached yet, encoded together (host encodings in parallel)
        {
            std::vector<std::string> keys;
            std::vector<std::vector<double>> dvs;
            for (auto &gg : groups)
                for (auto &bb : gg.second) {
                    const std::string fk = full_key(gg.first, bb.first);
                    if (m.pt_cache.count(fk)) continue;
                    std::vector<double> dv(slots, 0.0);
                    for (long d : bb.second) dv[(size_t)(((d + gg.first * pp.b1) % slots + slots) % slots)] = 1.0;
                    keys.push_back(fk);
                    dvs.push_back(std::move(dv));
                }
            std::vector<const std::vector<double> *> zp;
            for (auto &v : dvs) zp.push_back(&v);
            if (!zp.empty()) {
                std::vector<Pt> pts = c.vec_pts(zp, X(t, xd.level), t + 2);
                for (size_t i = 0; i < pts.size(); i++) m.pt_cache.emplace(keys[i], pts[i]);
            }
        }
        std::vector<Ct> rots = c.rotate_many(xd, babies, k);
        Ct z;
        bool have = false;
        for (auto &gg : groups) {
            const long g = gg.first;
            std::vector<std::pair<const Ct *, const Pt *>> terms;
            for (auto &bb : gg.second) {
                const Pt *pt = &m.pt_cache.at(full_key(g, bb.first));
                const size_t bi = std::lower_bound(babies.begin(), babies.end(), bb.first) - babies.begin();
                terms.push_back({&rots[bi], pt});
            }
            Ct inner = c.lincomb(terms, t);
            if (!have) {
                z = g ? c.rotate(inner, g * pp.b1, k) : inner;
                have = true;
            } else {
                z = g ? c.rotate_add(inner, g * pp.b1, z, k) : c.add(z, inner);
            }
        }
        return z;
    }

    // z <- z + rot(z, s) for s = period/2, ..., d
    Ct fold(Ct z, long d, long period)
    {
        for (long s = period / 2; s >= d; s /= 2) z = c.rotate_add(z, s, z, k);
        return z;
    }

    // both branches of the layer on one part's ciphertext, before the fold:
    // fused, one product with [W_f | W_b] of the bases plus the masked SiLU
    // values; otherwise W_f times the bases and W_b times the SiLU values of
    // x (the paper's two linear layers), both at the same level
    std::vector<Ct> part(const Ct &x, size_t li, size_t pc)
    {
        const LayerC &L = m.layers[li];
        const Part &P = L.parts[pc];
        const std::string tag =
            "L" + std::to_string(li) + "/" + (L.parts.size() > 1 ? "c" + std::to_string(pc) + "/" : "");
        const long slots = c.N / 2, nb = L.g + L.k;
        const int r = L.g + 2 * L.k + 1;
        Ct xr = li == 0 ? repeat_pack(x, P.n_blk, clog2i(L.g + 2 * L.k)) : x;
        // blocks of the input xr holds: the first layer's 2^ceil(log2(g+2k))
        // copies, or a periodic hidden input
        const long blocks = li == 0 ? pow2ceil(r - 1) : slots / P.n_blk;
        const bool shared = m.shared_cmp() && blocks >= r && (long)r * P.n_blk <= slots;
        Ct b = bspline(xr, L, P, tag, shared);
        if (m.fused()) {
            // SiLU on the repeat-packed input, masked to block g+k (the first
            // block the g+k bases leave free), added to the bases
            std::vector<double> mask(slots, 0.0);
            for (long i = 0; i < P.width; i++) mask[(size_t)nb * P.n_blk + i] = 1.0;
            tile(mask, L.period);
            Ct s = cheb_eval(xr, L.silu, L.silu_lo, L.silu_hi, &mask, tag + "S");
            int t = std::min(b.level, s.level) - 1;
            if (t < 0) throw HeError(-3, "layer does not fit the level budget");
            Ct z = c.add(c.mod_drop(b, t + 1), c.mod_drop(s, t + 1));
            return {matvec(z, SlotMatrix{P.W, L.n_out, nb + 1, P.n_in, P.n_blk, m.S}, L.d, t, L.period, tag + "W")};
        }
        Ct s = cheb_eval(x, L.silu, L.silu_lo, L.silu_hi, nullptr, tag + "S");
        if (m.naive()) {
            // no lazy combination: the bases permuted into row order, then W'
            if (b.level < 1) throw HeError(-3, "layer does not fit the level budget");
            Ct bp = permute(b, L, P, b.level - 1, tag + "P");
            const int t = std::min(bp.level, s.level) - 1;
            if (t < 0) throw HeError(-3, "layer does not fit the level budget");
            const long nq = (long)P.n_in * nb;
            Ct zr = matvec(bp, SlotMatrix{P.Wrow, L.n_out, 1, nq, nq * m.S, m.S}, L.d, t, L.period, tag + "Wr");
            Ct zb = matvec(s, SlotMatrix{P.Wb, L.n_out, 1, P.n_in, P.n_blk, m.S}, L.d, t, L.period, tag + "Wb");
            return {zr, zb};
        }
        int t = std::min(b.level, s.level) - 1;
        if (t < 0) throw HeError(-3, "layer does not fit the level budget");
        Ct zf = matvec(b, SlotMatrix{P.Wf, L.n_out, nb, P.n_in, P.n_blk, m.S}, L.d, t, L.period, tag + "Wf");
        Ct zb = matvec(s, SlotMatrix{P.Wb, L.n_out, 1, P.n_in, P.n_blk, m.S}, L.d, t, L.period, tag + "Wb");
        return {zf, zb};
    }

    // the parts' partial sums share one layout: add them (per product), then
    // fold each sum once; the layer output is the sum of the folded products
    Ct layer(const std::vector<Ct> &xs, size_t li)
    {
        const LayerC &L = m.layers[li];
        if (xs.size() != L.parts.size())
            throw HeError(-4, "layer " + std::to_string(li) + " takes " + std::to_string(L.parts.size()) +
                                  " input ciphertexts, got " + std::to_string(xs.size()));
        for (size_t pc = 1; pc < xs.size(); pc++)
            if (xs[pc].level != xs[0].level || xs[pc].nb != xs[0].nb)
                throw HeError(-1, "input ciphertexts differ in level or batch size");
        std::vector<Ct> z = part(xs[0], li, 0);
        for (size_t pc = 1; pc < xs.size(); pc++) {
            std::vector<Ct> zc = part(xs[pc], li, pc);
            for (size_t j = 0; j < z.size(); j++) z[j] = c.add(z[j], zc[j]);
        }
        Ct y = fold(z[0], L.d * m.S, L.period);
        for (size_t j = 1; j < z.size(); j++) y = c.add(y, fold(z[j], L.d * m.S, L.period));
        return y;
    }
};

Ct eval_layer(Ctx &c, Model &m, const Keys &k, const std::vector<Ct> &in, size_t li)
{
    Eval e(c, k, m);
    return e.layer(in, li);
}

Ct cheb_series(Ctx &c, const Keys &k, const Ct &x, const std::vector<double> &cf, double lo, double hi)
{
    Model none;
    Eval e(c, k, none);
    return e.cheb_eval(x, cf, lo, hi);
}

Ct eval_model(Ctx &c, Model &m, const Keys &k, const std::vector<Ct> &in)
{
    if (m.refresh && m.layers.size() > 1)
        throw HeError(-7, "model compiled with refresh between layers: evaluate layer by layer");
    Eval e(c, k, m);
    Ct x = e.layer(in, 0);
    for (size_t li = 1; li < m.layers.size(); li++) x = e.layer({x}, li);
    return x;
}

}  // namespace hk
