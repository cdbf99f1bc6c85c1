// Device-resident RNS-CKKS operations (Preliminaries, Homomorphic Encryption:
// add, subtract, multiply, rotate), orchestrated on one HIP stream.
#include "ckks.hpp"

#include <algorithm>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>

namespace hk {

// ------------------------------------------------------------------- memory
// Allocation sizes are rounded up to size classes (256 B granules up to
// 1 MiB, then eighths of the power of two below the size: at most 12.5% more)
// so that buffers freed by a batch of one size serve batches of nearby sizes.
static size_t size_class(size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes <= ((size_t)1 << 20)) return bytes;
    size_t p = (size_t)1 << (63 - __builtin_clzll(bytes));
    const size_t g = p >> 3;
    return (bytes + g - 1) / g * g;
}

void *Pool::get(size_t bytes)
{
    bytes = size_class(bytes);
    void *p = nullptr;
    if (hold) {
        auto h = hold->find(bytes);
        if (h != hold->end()) {
            p = h->second;
            hold->erase(h);
            live += bytes;
            peak = std::max(peak, live);
            return p;
        }
    }
    auto it = free_.find(bytes);
    if (it != free_.end()) {
        p = it->second;
        free_.erase(it);
        cached -= bytes;
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            trim();
            if (hipMalloc(&p, bytes) != hipSuccess) {
                (void)hipGetLastError();
                throw HeError(-2, "device allocation of " + std::to_string(bytes) + " bytes failed");
            }
        }
    }
    live += bytes;
    peak = std::max(peak, live);
    return p;
}

void Pool::put(void *p, size_t bytes)
{
    bytes = size_class(bytes);
    live -= bytes;
    if (hold) {
        hold->emplace(bytes, p);
        return;
    }
    cached += bytes;
    free_.emplace(bytes, p);
}

void Pool::trim()
{
    for (auto &kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached = 0;
}

Pool::~Pool() { trim(); }

DevBuf::~DevBuf() { ctx->pool.put(p, words * sizeof(u64)); }

Buf Ctx::alloc(size_t words)
{
    u64 *p = (u64 *)pool.get(words * sizeof(u64));
    return Buf(new DevBuf{this, p, words});
}

void Ctx::upload(u64 *dst, const u64 *src, size_t words)
{
    HIP_CHECK(hipMemcpyAsync(dst, src, words * sizeof(u64), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
}

void Ctx::download(u64 *dst, const u64 *src, size_t words)
{
    HIP_CHECK(hipMemcpyAsync(dst, src, words * sizeof(u64), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
}

void Ctx::sync() { HIP_CHECK(hipStreamSynchronize(st)); }

// ------------------------------------------------------------- kernel timer
void KernelTimer::before(hipStream_t s)
{
    if (used == cap) {
        size_t ncap = cap ? 2 * cap : 1024;
        Rec *n = new Rec[ncap];
        for (size_t i = 0; i < cap; i++) n[i] = recs[i];
        for (size_t i = cap; i < ncap; i++) {
            HIP_CHECK(hipEventCreate(&n[i].a));
            HIP_CHECK(hipEventCreate(&n[i].b));
        }
        delete[] recs;
        recs = n;
        cap = ncap;
    }
    HIP_CHECK(hipEventRecord(recs[used].a, s));
}

void KernelTimer::after(hipStream_t s, double bytes, double ops)
{
    HIP_CHECK(hipEventRecord(recs[used].b, s));
    recs[used].bytes = bytes;
    recs[used].ops = ops;
    used++;
}

void Ctx::profile(int kernel_id)
{
    sync();
    timer.target = kernel_id;
    timer.used = 0;
}

void Ctx::profile_read(double &ms, u64 &launches, double &bytes, double &ops)
{
    sync();
    ms = bytes = ops = 0;
    for (size_t i = 0; i < timer.used; i++) {
        float t = 0;
        HIP_CHECK(hipEventElapsedTime(&t, timer.recs[i].a, timer.recs[i].b));
        ms += t;
        bytes += timer.recs[i].bytes;
        ops += timer.recs[i].ops;
    }
    launches = timer.used;
}

// ------------------------------------------------------------------ context
Ctx::Ctx(int logN_, int L_, int scale_bits, int base_bits, int alpha_, int special_bits, int w_, double sigma_,
         hipStream_t stream, bool integer_words, int boot_levels, int boot_bits, int hamming_)
    : logN(logN_), N(1 << logN_), L(L_), alpha(alpha_), w(w_), L1(L_ + 1), top(L_ - boot_levels), hamming(hamming_),
      sigma(sigma_)
{
    make_chain(logN, base_bits, L, scale_bits, alpha, special_bits, boot_levels, boot_bits, q, p, S);
    mods = q;
    mods.insert(mods.end(), p.begin(), p.end());
    if (stream) {
        st = (hipStream_t)stream;
    } else {
        HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own_stream = true;
    }
    const int np = (int)mods.size();
    pc.resize(np);
    for (int i = 0; i < np; i++) {
        u64 m = mods[i];
        PrimeConst &c = pc[i];
        std::memset(&c, 0, sizeof(c));
        c.q = m;
        c.bits = 64 - __builtin_clzll(m);
        c.mu = (u64)(((u128)1 << (2 * c.bits)) / m);
        // -q^-1 mod 2^64 by Newton iteration
        u64 inv = 1;
        for (int k = 0; k < 7; k++) inv *= 2 - m * inv;
        c.qinv_neg = (u64)0 - inv;
        c.r1 = (u64)(((u128)1 << 64) % m);
        c.r1p = shoup_of(c.r1, m);
        c.ninv = hinv((u64)N % m, m);
        c.ninvp = shoup_of(c.ninv, m);
        c.fp = c.bits <= 46 && !integer_words;
        c.qd = (double)m;
        c.qinvd = 1.0 / (double)m;
        const u64 r32 = (u64)(((u128)1 << 32) % m);
        c.r32d = (double)r32;
        c.r32c = (double)r32 / (double)m;
    }
    fp_lo = pc[0].fp ? 0 : 1;
    fp_top = 0;
    while (fp_top + 1 <= L && pc[fp_top + 1].fp) fp_top++;
    ks_fused = fp_top >= 1;
    d_pc_buf = alloc((sizeof(PrimeConst) * np + 7) / 8);
    HIP_CHECK(hipMemcpyAsync(d_pc_buf->p, pc.data(), sizeof(PrimeConst) * np, hipMemcpyHostToDevice, st));
    d_pc = (const PrimeConst *)d_pc_buf->p;
    // twiddles: psi^brv(k) and psi^-brv(k) with Shoup companions
    std::vector<u64> tw((size_t)4 * np * N);
    std::vector<TwF> twf((size_t)2 * np * N);
    for (int i = 0; i < np; i++) {
        u64 m = mods[i];
        u64 psi = primitive_2n_root(m, logN), ipsi = hinv(psi, m);
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; k++) {
            pw[k] = hmul(pw[k - 1], psi, m);
            ipw[k] = hmul(ipw[k - 1], ipsi, m);
        }
        u64 *fw = &tw[(size_t)(0 * np + i) * N], *fwp = &tw[(size_t)(1 * np + i) * N];
        u64 *iw = &tw[(size_t)(2 * np + i) * N], *iwp = &tw[(size_t)(3 * np + i) * N];
        for (int k = 0; k < N; k++) {
            u32 r = 0;
            for (int b = 0; b < logN; b++)
                if (k >> b & 1) r |= 1u << (logN - 1 - b);
            fw[k] = pw[r];
            fwp[k] = shoup_of(fw[k], m);
            iw[k] = ipw[r];
            iwp[k] = shoup_of(iw[k], m);
            twf[(size_t)i * N + k] = TwF{(double)fw[k], (double)fw[k] / (double)m};
            twf[(size_t)(np + i) * N + k] = TwF{(double)iw[k], (double)iw[k] / (double)m};
        }
    }
    twf_buf = alloc(twf.size() * 2);
    upload(twf_buf->p, (const u64 *)twf.data(), twf.size() * 2);
    T.ffw = (const TwF *)twf_buf->p;
    T.fiw = (const TwF *)twf_buf->p + (size_t)np * N;
    // factored second-pass twiddles (LC = 8 stages over rows of 256 words)
    {
        const int LR = logN - 8, rows = 1 << LR;
        std::vector<TwF> ab((size_t)2 * np * ((size_t)rows * 8 + 256), TwF{0.0, 0.0});
        for (int dir = 0; dir < 2; dir++)
            for (int i = 0; i < np; i++) {
                const u64 m = mods[i];
                const u64 *W = &tw[(size_t)((dir == 0 ? 0 : 2) * np + i) * N];
                TwF *A = &ab[((size_t)dir * np + i) * rows * 8];
                TwF *B = &ab[(size_t)2 * np * rows * 8 + ((size_t)dir * np + i) * 256];
                for (int sp = 0; sp < 8; sp++) {
                    const size_t base = (size_t)1 << (LR + sp);
                    for (int r = 0; r < rows; r++) {
                        const u64 a = W[base + ((size_t)r << sp)];
                        A[(size_t)r * 8 + sp] = TwF{(double)a, (double)a / (double)m};
                    }
                    const u64 inv0 = hinv(W[base], m);
                    for (int u = 0; u < (1 << sp); u++) {
                        const u64 b = hmul(W[base + u], inv0, m);
                        B[(1 << sp) - 1 + u] = TwF{(double)b, (double)b / (double)m};
                    }
                }
            }
        twab_buf = alloc(ab.size() * 2);
        upload(twab_buf->p, (const u64 *)ab.data(), ab.size() * 2);
        const TwF *abp = (const TwF *)twab_buf->p;
        T.fa = abp;
        T.ia = abp + (size_t)np * rows * 8;
        T.fb = abp + (size_t)2 * np * rows * 8;
        T.ib = T.fb + (size_t)np * 256;
    }
    tw_buf = alloc(tw.size());
    upload(tw_buf->p, tw.data(), tw.size());
    T.pc = d_pc;
    T.fw = tw_buf->p;
    T.fwp = tw_buf->p + (size_t)np * N;
    T.iw = tw_buf->p + (size_t)2 * np * N;
    T.iwp = tw_buf->p + (size_t)3 * np * N;
    T.logN = logN;
    // P^-1 mod q_i
    std::vector<u64> pv(2 * (L + 1));
    for (int i = 0; i <= L; i++) {
        u64 P = 1;
        for (u64 pj : p) P = hmul(P, pj % q[i], q[i]);
        pv[i] = hinv(P, q[i]);
        pv[L + 1 + i] = shoup_of(pv[i], q[i]);
    }
    // then the same values as FP64 pairs (value, value / q_i)
    pv.resize(4 * (L + 1));
    for (int i = 0; i <= L; i++) {
        const double w = (double)pv[i], c = w / (double)q[i];
        std::memcpy(&pv[2 * (L + 1) + 2 * i], &w, 8);
        std::memcpy(&pv[2 * (L + 1) + 2 * i + 1], &c, 8);
    }
    pinv = alloc(pv.size());
    upload(pinv->p, pv.data(), pv.size());
    // P mod q_i, Shoup words and FP64 pairs (value, value / q_i): the rescale
    // term of the merged ModDown
    std::vector<u64> pmv(4 * (L + 1));
    for (int i = 0; i <= L; i++) {
        u64 P = 1;
        for (u64 pj : p) P = hmul(P, pj % q[i], q[i]);
        pmv[i] = P;
        pmv[L + 1 + i] = shoup_of(P, q[i]);
        const double w = (double)P, c = w / (double)q[i];
        std::memcpy(&pmv[2 * (L + 1) + 2 * i], &w, 8);
        std::memcpy(&pmv[2 * (L + 1) + 2 * i + 1], &c, 8);
    }
    pmod = alloc(pmv.size());
    upload(pmod->p, pmv.data(), pmv.size());
    // ModDown constants: P-limb INTT scale (P/p_k)^-1 N^-1 mod p_k, and
    // (P/p_k) mod q_i in Montgomery form
    std::vector<u64> md(2 * alpha + (size_t)alpha * (L + 1));
    for (int k = 0; k < alpha; k++) {
        u64 pk = p[k], h = 1;
        for (int k2 = 0; k2 < alpha; k2++)
            if (k2 != k) h = hmul(h, p[k2] % pk, pk);
        u64 sc = hmul(hinv(h, pk), hinv((u64)N % pk, pk), pk);
        md[k] = sc;
        md[alpha + k] = shoup_of(sc, pk);
        for (int i = 0; i <= L; i++) {
            u64 hq = 1;
            for (int k2 = 0; k2 < alpha; k2++)
                if (k2 != k) hq = hmul(hq, p[k2] % q[i], q[i]);
            md[2 * alpha + (size_t)k * (L + 1) + i] = (u64)(((u128)hq << 64) % q[i]);
        }
    }
    md_tab = alloc(md.size());
    upload(md_tab->p, md.data(), md.size());
    // the entry points that allocate nothing: every level's rescale table now,
    // and this device's scratch address
    for (int l = 1; l <= L; l++) (void)rescale_table(l, 1);
    scratch = noalloc_scratch_setup();
}

Ctx::~Ctx()
{
    try {
        if (st) (void)hipStreamSynchronize(st);
    } catch (...) {
    }
    for (size_t i = 0; i < timer.cap; i++) {
        (void)hipEventDestroy(timer.recs[i].a);
        (void)hipEventDestroy(timer.recs[i].b);
    }
    delete[] timer.recs;
    ks_cache.clear();
    md_tab.reset();
    rescale_inv.clear();
    rescale_add.clear();
    const_cache.clear();
    const_plain_cache.clear();
    int_cache.clear();
    pinv.reset();
    pmod.reset();
    tw_buf.reset();
    twf_buf.reset();
    twab_buf.reset();
    d_pc_buf.reset();
    pool.trim();
    if (own_stream && st) (void)hipStreamDestroy(st);
}

u64 Ctx::galois_elt(long step) const
{
    if (step == kStepConjugate) return 2ull * N - 1;
    long slots = N / 2;
    long t = ((step % slots) + slots) % slots;
    return hpow(5, (u64)t, 2ull * N);
}

void Ctx::ntt(PolySet ps, LimbMap lm, bool inverse, int skip_lo, int skip_hi)
{
    launch_ntt(T, ps, lm, skip_lo, skip_hi, inverse, st, &timer);
    n_launch += 2;
}

PolySet Ctx::ctset(const Ct &c, int nl) const
{
    return PolySet{c.d(), 2l * N * c.nb, (long)N, nl < 0 ? c.level + 1 : nl, 2 * c.nb};
}

PolySet Ctx::c0set(const Ct &c) const { return PolySet{c.d(), 2l * N * c.nb, 2l * N, c.level + 1, c.nb}; }

// ------------------------------------------------------------ simple ct ops
Ct Ctx::new_ct(int level, int nb)
{
    Ct c;
    c.level = level;
    c.nb = nb;
    c.buf = alloc((size_t)(level + 1) * 2 * N * nb);
    return c;
}

Ct Ctx::add(const Ct &a, const Ct &b)
{
    if (a.level != b.level || a.nb != b.nb) throw HeError(-1, "add: level mismatch");
    Ct o = new_ct(a.level, a.nb);
    launch_addsub(d_pc, ctset(o), ctset(a), ctset(b), lmap(a.level + 1), 0, N, st);
    n_launch++;
    return o;
}

Ct Ctx::sub(const Ct &a, const Ct &b)
{
    if (a.level != b.level || a.nb != b.nb) throw HeError(-1, "sub: level mismatch");
    Ct o = new_ct(a.level, a.nb);
    launch_addsub(d_pc, ctset(o), ctset(a), ctset(b), lmap(a.level + 1), 1, N, st);
    n_launch++;
    return o;
}

const Buf &Ctx::int_factor(long k)
{
    auto it = int_cache.find((int)k);
    if (it == int_cache.end()) {
        std::vector<u64> v(2 * (L + 1));
        for (int i = 0; i <= L; i++) {
            long r = k % (long)q[i];
            v[i] = r < 0 ? (u64)(r + (long)q[i]) : (u64)r;
            v[L + 1 + i] = shoup_of(v[i], q[i]);
        }
        Buf b = alloc(v.size());
        upload(b->p, v.data(), v.size());
        it = int_cache.emplace((int)k, b).first;
    }
    return it->second;
}

Ct Ctx::mul_int(const Ct &a, long k)
{
    const Buf &f = int_factor(k);
    Ct o = new_ct(a.level, a.nb);
    launch_mul_scalar(d_pc, ctset(o), ctset(a), f->p, f->p + L + 1, lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

Ct Ctx::affine(const Ct &a, long k, const double *c, const Buf *pt)
{
    const u64 *kf = nullptr, *kfp = nullptr;
    if (k != 1) {
        const Buf &f = int_factor(k);
        kf = f->p;
        kfp = f->p + L + 1;
    }
    const u64 *cr = c ? const_residues(*c, S[a.level]) : nullptr;
    Ct o = new_ct(a.level, a.nb);
    launch_add_c0(d_pc, ctset(o), ctset(a), kf, kfp, cr, pt ? (*pt)->p : nullptr, lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

// residues over every Q prime of the constant c encoded at scale sc (cached)
const u64 *Ctx::const_residues(double c, double sc)
{
    u64 kc, ks;
    std::memcpy(&kc, &c, 8);
    std::memcpy(&ks, &sc, 8);
    auto key = std::make_pair(kc, ks);
    auto it = const_cache.find(key);
    if (it == const_cache.end()) {
        std::vector<u64> v(L + 1);
        encode_const_rns(c, sc, q.data(), L + 1, v.data());
        Buf b = alloc(v.size());
        upload(b->p, v.data(), v.size());
        it = const_cache.emplace(key, b).first;
    }
    return it->second->p;
}

Ct Ctx::add_const(const Ct &a, double c)
{
    const u64 *cr = const_residues(c, S[a.level]);
    Ct o = new_ct(a.level, a.nb);
    launch_add_c0(d_pc, ctset(o), ctset(a), nullptr, nullptr, cr, nullptr, lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

Ct Ctx::add_plain(const Ct &a, const Buf &pt)
{
    Ct o = new_ct(a.level, a.nb);
    launch_add_c0(d_pc, ctset(o), ctset(a), nullptr, nullptr, nullptr, pt->p, lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

Ct Ctx::mod_drop(const Ct &a, int l) const
{
    if (l > a.level || l < 0) throw HeError(-1, "mod_drop: bad level");
    Ct o = a;
    o.level = l;
    return o;
}

Ct Ctx::mod_raise(const Ct &a)
{
    if (a.level != 0) throw HeError(-1, "mod_raise: the input must be at level 0");
    const int np = 2 * a.nb;
    Buf tmp = alloc((size_t)np * N);
    PolySet t{tmp->p, (long)np * N, (long)N, 1, np};
    launch_copy(t, PolySet{a.d(), 2l * N * a.nb, (long)N, 1, np}, N, st);
    ntt(t, lmap(1), true);
    Ct o = new_ct(L, a.nb);
    launch_modraise(d_pc, ctset(o), tmp->p, lmap(L + 1), N, st);
    ntt(ctset(o), lmap(L + 1), false);
    n_launch += 2;
    return o;
}

Ct Ctx::mul_i(const Ct &a)
{
    if (!mono_half) {
        std::vector<u64> h((size_t)(L + 1) * N, 0);
        for (int t = 0; t <= L; t++) h[(size_t)t * N + N / 2] = 1;
        mono_half = alloc(h.size());
        upload(mono_half->p, h.data(), h.size());
        ntt(PolySet{mono_half->p, (long)N, 0, L + 1, 1}, lmap(L + 1), false);
    }
    Ct o = new_ct(a.level, a.nb);
    launch_pmul(d_pc, ctset(o), ctset(a), PolySet{mono_half->p, (long)N, 0, a.level + 1, 2 * a.nb},
                lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

// ------------------------------------------------------------------ rescale
const Buf &Ctx::rescale_table(int l, long k)
{
    auto it = rescale_inv.find(std::make_pair(l, k));
    if (it != rescale_inv.end()) return it->second;
    // [l] k q_l^-1 mod q_i, [l] Shoup words, [l] FP64 pairs (value, value / q_i)
    std::vector<u64> v(4 * l);
    for (int i = 0; i < l; i++) {
        const long r = k % (long)q[i];
        const u64 km = r < 0 ? (u64)(r + (long)q[i]) : (u64)r;
        v[i] = hmul(hinv(q[l] % q[i], q[i]), km, q[i]);
        v[l + i] = shoup_of(v[i], q[i]);
        const double w = (double)v[i], c = w / (double)q[i];
        std::memcpy(&v[2 * l + 2 * i], &w, 8);
        std::memcpy(&v[2 * l + 2 * i + 1], &c, 8);
    }
    Buf b = alloc(std::max<size_t>(v.size(), 1));
    if (l) upload(b->p, v.data(), v.size());
    return rescale_inv.emplace(std::make_pair(l, k), b).first->second;
}

// Rescale with rounding (divide by q_l, drop limb l): the dropped limb goes to
// coefficient form; the forward transforms of ([c_l + h] - h) mod q_i and the
// final (c_i - t_i) q_l^-1 run inside one fused NTT.
Ct Ctx::rescale(const Ct &a) { return rescale_affine(a, 1, nullptr); }

Ct Ctx::rescale_const_mul(const Ct &a, const Pt &pt, int t, const double *c)
{
    const int l = t + 1, np = 2 * a.nb;
    if (l < 1 || a.level < l) throw HeError(-3, "rescale_const_mul: operand below target + 1");
    n_rescale++;
    const u64 *w = pt.plain->p;
    const long P = L + 1;
    Buf last = alloc((size_t)np * N);
    // limb l of C a in coefficient form: C_l N^-1 applied to the inverse transform of a's limb l
    launch_intt_from(T, PolySet{last->p, (long)N, (long)N, 1, np}, LimbMap{1, L1, l},
                     a.d() + (size_t)l * 2 * N * a.nb, 2l * N * a.nb, (long)N, 0, w + 2 * P + l, w + 3 * P + l, st,
                     &timer);
    Buf tmp = alloc((size_t)l * np * N);
    Ct o = new_ct(l - 1, a.nb);
    const Buf &inv = rescale_table(l, 1);
    const u64 *cadd = c ? rescale_addend(l, 1, *c) : nullptr;
    launch_rescale_ntt(T, tmp->p, l, np, last->p, q[l], a.d(), 2l * N * a.nb, (long)N, o.d(), 2l * N * a.nb,
                       (long)N, inv->p, inv->p + l, (const TwF *)(inv->p + 2 * l), w, w + P, cadd, L1, st, &timer);
    n_launch += 4;
    return o;
}

// per limb i < l: the constant c at scale S[l-1] divided by k q_l^-1 (mod q_i), so
// that adding it before the rescale's final product adds c to the result
const u64 *Ctx::rescale_addend(int l, long k, double c)
{
    u64 kc;
    std::memcpy(&kc, &c, 8);
    auto key = std::make_tuple(l, k, kc);
    auto it = rescale_add.find(key);
    if (it != rescale_add.end()) return it->second->p;
    std::vector<u64> cr(L + 1), v(std::max(l, 1), 0);
    encode_const_rns(c, S[l - 1], q.data(), L + 1, cr.data());
    for (int i = 0; i < l; i++) {
        const long r = k % (long)q[i];
        const u64 km = r < 0 ? (u64)(r + (long)q[i]) : (u64)r;
        if (km == 0) throw HeError(-1, "rescale: factor divisible by a prime");
        v[i] = hmul(hmul(cr[i], q[l] % q[i], q[i]), hinv(km, q[i]), q[i]);
    }
    Buf b = alloc(v.size());
    upload(b->p, v.data(), v.size());
    return rescale_add.emplace(key, b).first->second->p;
}

// the dropped limb to coefficient form (into last, np N words), then the
// fused transforms of the rescale (intermediate in tmp, l np N words) into o
static void rescale_launch(Ctx &c, const Ct &a, Ct &o, const Buf &inv, const u64 *cadd, u64 *last, u64 *tmp)
{
    const int l = a.level, np = 2 * a.nb;
    const long N = c.N;
    c.n_rescale++;
    launch_intt_from(c.T, PolySet{last, N, N, 1, np}, LimbMap{1, c.L1, l}, a.d() + (size_t)l * 2 * N * a.nb,
                     2l * N * a.nb, N, 0, nullptr, nullptr, c.st, &c.timer);
    launch_rescale_ntt(c.T, tmp, l, np, last, c.q[l], a.d(), 2l * N * a.nb, N, o.d(), 2l * N * a.nb, N, inv->p,
                       inv->p + l, (const TwF *)(inv->p + 2 * l), nullptr, nullptr, cadd, c.L1, c.st, &c.timer);
    c.n_launch += 4;
}

Ct Ctx::rescale_affine(const Ct &a, long k, const double *c)
{
    const int l = a.level, np = 2 * a.nb;
    if (l < 1) throw HeError(-3, "rescale: no level left");
    Buf last = alloc((size_t)np * N);
    Buf tmp = alloc((size_t)l * np * N);
    Ct o = new_ct(l - 1, a.nb);
    const Buf &inv = rescale_table(l, k);
    const u64 *cadd = c ? rescale_addend(l, k, *c) : nullptr;
    rescale_launch(*this, a, o, inv, cadd, last->p, tmp->p);
    return o;
}

void Ctx::rescale_into(const Ct &a, Ct &o, u64 *scr)
{
    const int l = a.level;
    if (l < 1) throw HeError(-3, "rescale: no level left");
    if (a.nb != 1 || o.nb != 1 || o.level != l - 1) throw HeError(-1, "rescale_into: shapes do not match");
    auto it = rescale_inv.find(std::make_pair(l, 1l));
    if (it == rescale_inv.end()) throw HeError(-7, "rescale_into: no table for this level");
    rescale_launch(*this, a, o, it->second, nullptr, scr, scr + (size_t)2 * N);
}

// ----------------------------------------------------------- key switching
const KsTable &Ctx::ks_table(int l)
{
    auto it = ks_cache.find(l);
    if (it != ks_cache.end()) return it->second;
    const int nq = l + 1, next = nq + alpha, nd = ndig(l);
    std::vector<u64> v(2 * (size_t)nq + (size_t)nd * w * next, 0);
    std::vector<TwF> vf((size_t)nd * w * next + nq, TwF{0.0, 0.0});
    LimbMap lm = lmap(nq);
    KsTable kt;
    kt.wide[0] = kt.wide[1] = 0;
    kt.dbl[0] = kt.dbl[1] = 0;
    for (int j = 0; j < nd; j++) {
        const int lo = j * w, hi = std::min(lo + w, nq);
        for (int i = lo; i < hi; i++) {
            u64 h = 1;
            for (int k = lo; k < hi; k++)
                if (k != i) h = hmul(h, q[k] % q[i], q[i]);
            u64 sc = hmul(hinv(h, q[i]), hinv((u64)N % q[i], q[i]), q[i]);
            v[i] = sc;
            v[nq + i] = shoup_of(sc, q[i]);
            if (64 - __builtin_clzll(q[i]) > 50) kt.wide[j / 8] |= 1ull << (8 * (j % 8) + (i - lo));
            if (pc[i].fp) {
                kt.dbl[j / 8] |= 1ull << (8 * (j % 8) + (i - lo));
                vf[(size_t)nd * w * next + i] = TwF{(double)sc, (double)sc / (double)q[i]};
            }
            for (int t = 0; t < next; t++) {
                if (t >= lo && t < hi) continue;
                u64 m = mods[lm.prime(t)], hm = 1;
                for (int k = lo; k < hi; k++)
                    if (k != i) hm = hmul(hm, q[k] % m, m);
                const size_t o = ((size_t)j * w + (i - lo)) * next + t;
                v[2 * (size_t)nq + o] = (u64)(((u128)hm << 64) % m);
                if (pc[lm.prime(t)].fp) vf[o] = TwF{(double)hm, (double)hm / (double)m};
            }
        }
    }
    kt.fbuf = alloc(vf.size() * 2);
    upload(kt.fbuf->p, (const u64 *)vf.data(), vf.size() * 2);
    kt.hatf = (const TwF *)kt.fbuf->p;
    kt.scalef = kt.hatf + (size_t)nd * w * next;
    kt.buf = alloc(v.size());
    upload(kt.buf->p, v.data(), v.size());
    kt.scale = kt.buf->p;
    kt.scalep = kt.buf->p + nq;
    kt.hatm = kt.buf->p + 2 * nq;
    return ks_cache.emplace(l, kt).first->second;
}

// Hybrid key switching (Han-Ki): d is split into digits of w Q limbs; each
// digit is extended to Q_l u P by fast basis conversion (ModUp), multiplied by
// the key digit and accumulated; the sum is divided by P (ModDown).  For a
// rotation the Galois automorphism acts on the extended digits; because the
// Galois keys are stored permuted by sigma^-1, the inner product runs
// unpermuted and sigma is applied when ModDown reads the accumulator.
Ctx::ModUp Ctx::modup(const u64 *d, long ls, long es, int l, int nb)
{
    ModUp m;
    m.d = d;
    m.ls = ls;
    m.es = es;
    m.l = l;
    m.nb = nb;
    const int nq = l + 1, next = nq + alpha, nd = ndig(l);
    const LimbMap lm = lmap(nq);
    const KsTable &kt = ks_table(l);
    // y = INTT(d) * invhat / N, then every digit's conversion and NTT
    Buf y = alloc((size_t)nb * nq * N);
    launch_intt_modup(T, PolySet{y->p, (long)N, (long)nq * N, nq, nb}, lm, d, ls, es, kt.scale, kt.scalep,
                      kt.scalef, st, &timer);
    m.ext = alloc((size_t)nb * nd * next * N);
    launch_modup(T, m.ext->p, nd, nq, alpha, w, nb, lm, y->p, kt.hatm, kt.hatf, kt.wide, kt.dbl, st, &timer);
    n_launch += 3;
    return m;
}

Buf Ctx::inner_product(const ModUp &m, const SwitchKey &key)
{
    n_ks += m.nb;
    const int l = m.l, nb = m.nb, nq = l + 1, next = nq + alpha, nd = ndig(l), ktot = L + 1 + alpha;
    const LimbMap lm = lmap(nq);
    Buf acc = alloc((size_t)nb * 2 * next * N);
    if (launch_keyip(d_pc, acc->p, (long)next * N, 2l * next * N, m.ext->p, (long)next * N, (long)nd * next * N,
                     m.d, m.ls, m.es, key.buf->p, 2l * ktot * N, (long)ktot * N, nd, next, 0, 0, nq, w, nb, lm, L1,
                     logN, st, &timer) != 0)
        throw HeError(-1, "key switch: " + std::to_string(nd) + " digits (at most 16 supported)");
    n_launch++;
    return acc;
}

void Ctx::keyswitch_from(const ModUp &m, const SwitchKey &key, u64 galois, const u64 *base, long base_ls,
                         long base_es, int base_mask, Ct &out, const Ct *addend)
{
    Buf acc = inner_product(m, key);
    moddown_into(acc, m.l, m.nb, galois, base, base_ls, base_es, base_mask, out, addend);
}

void Ctx::moddown_into(const Buf &acc, int l, int nb, u64 galois, const u64 *base, long base_ls, long base_es,
                       int base_mask, Ct &out, const Ct *addend)
{
    const int nq = l + 1, next = nq + alpha;
    const LimbMap lm = lmap(nq);
    // ModDown of the 2 nb accumulator polynomials
    Buf yP = alloc((size_t)nb * 2 * alpha * N);
    launch_intt_from(T, PolySet{yP->p, (long)N, (long)alpha * N, alpha, 2 * nb}, LimbMap{0, L1},
                     acc->p + (size_t)nq * N, (long)N, (long)next * N, galois, md_tab->p, md_tab->p + alpha, st,
                     &timer);
    Buf tmp = alloc((size_t)nb * 2 * nq * N);
    OutModdownArgs oa{acc->p, (long)N, (long)next * N, base, base_ls, base_es, (long)N, base_mask, galois, out.d(),
                      2l * N * nb, (long)N, pinv->p, pinv->p + L + 1};
    oa.pinvf = (const TwF *)(pinv->p + 2 * (L + 1));
    if (addend) {
        if (addend->level != l || addend->nb != nb) throw HeError(-1, "rotate_add: operand shapes differ");
        oa.add = addend->d();
        oa.als = 2l * N * nb;
        oa.aes = 2l * N;
    }
    launch_moddown(T, tmp->p, nq, alpha, 2 * nb, lm, yP->p, md_tab->p + 2 * alpha, L + 1, oa, st, &timer);
    n_launch += 5;
}

// Hybrid key switching (Han-Ki): d is split into digits of w Q limbs; each
// digit is extended to Q_l u P by fast basis conversion (ModUp), multiplied by
// the key digit and accumulated; the sum is divided by P (ModDown).  For a
// rotation the Galois automorphism acts on the extended digits; because the
// Galois keys are stored permuted by sigma^-1, the inner product runs
// unpermuted and sigma is applied when ModDown reads the accumulator.
// d: nb polynomials, limb stride ls, element stride es.
void Ctx::keyswitch(const u64 *d, long ls, long es, int l, int nb, const SwitchKey &key, u64 galois,
                    const u64 *base, long base_ls, long base_es, int base_mask, Ct &out, const Ct *addend)
{
    Buf acc = keyswitch_acc(d, ls, es, l, nb, key);
    moddown_into(acc, l, nb, galois, base, base_ls, base_es, base_mask, out, addend);
}

// ModUp and the key inner product of a key switch: the accumulators
// [nb][2][l+1+alpha][N], before ModDown
Buf Ctx::keyswitch_acc(const u64 *d, long ls, long es, int l, int nb, const SwitchKey &key)
{
    // the configuration chosen for this (level, batch), by default fused with spans of 8
    auto tc = ks_tune.find(std::make_pair(l, nb));
    const int cfg = tc == ks_tune.end() ? 8 : tc->second;
    // the fused kernel handles q_fp_lo..q_min(l, fp_top); level 0 takes the
    // separate path
    if (!ks_fused || !key.fbuf || l == 0 || cfg == 0) return inner_product(modup(d, ls, es, l, nb), key);
    // ModUp with the inner product fused into the second pass on the FP64
    // limbs [fp_lo, fp_hi); the extended digits are stored only on the other
    // limbs (q_0 below fp_lo, the limbs from fp_hi up, the special primes),
    // whose inner product follows separately
    n_ks += nb;
    const int nq = l + 1, next = nq + alpha, nd = ndig(l), ktot = L + 1 + alpha;
    const int fp_hi = std::min(nq, fp_top + 1), n_out = fp_lo + (nq - fp_hi);
    if (nd > 16) throw HeError(-1, "key switch: " + std::to_string(nd) + " digits (at most 16 supported)");
    const LimbMap lm = lmap(nq);
    const KsTable &kt = ks_table(l);
    Buf y = alloc((size_t)nb * nq * N);
    launch_intt_modup(T, PolySet{y->p, (long)N, (long)nq * N, nq, nb}, lm, d, ls, es, kt.scale, kt.scalep,
                      kt.scalef, st, &timer);
    Buf ext = alloc((size_t)nb * nd * next * N);
    Buf acc = alloc((size_t)nb * 2 * next * N);
    ModupKeyipArgs a{fp_lo, fp_hi, n_out, nb, d, ls, es, (const double *)key.fbuf->p, 2l * ktot * N,
                     (long)ktot * N, acc->p, 2l * next * N, (long)next * N, cfg};
    launch_modup_keyip(T, ext->p, nd, nq, alpha, w, nb, lm, y->p, kt.hatm, kt.hatf, kt.wide, kt.dbl, a, st, &timer);
    y.reset();
    launch_keyip(d_pc, acc->p, (long)next * N, 2l * next * N, ext->p, (long)next * N, (long)nd * next * N, d, ls, es,
                 key.buf->p, 2l * ktot * N, (long)ktot * N, nd, n_out + alpha, fp_lo, fp_hi, nq, w, nb, lm, L1, logN,
                 st, &timer);
    ext.reset();
    n_launch += 6;
    return acc;
}

// Key-switch autotuner: for one batch size, at every level, times ModUp and
// the key inner product (the part whose kernels differ) in each configuration
// (0: ModUp, then the inner product over every limb; 1, 8, 32: the fused
// kernel with block spans of that many groups) on a zero input, median of
// `reps` runs after one warm-up, and keeps the fastest.  Every configuration
// computes the same residues.  Synchronises the stream: not for use while a
// graph is being captured.
std::vector<int> Ctx::autotune_keyswitch(const SwitchKey &key, int nb, int reps)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_CHECK(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) throw HeError(-7, "autotune: the stream is being captured");
    std::vector<int> chosen(L + 1, 8);
    const int cands[4] = {0, 1, 8, 32};
    // one zero input for every level (element stride (l+1) N within it)
    const size_t words = (size_t)nb * (L + 1) * N;
    Buf d = alloc(words);
    {
        std::vector<u64> z(words, 0);
        upload(d->p, z.data(), words);
    }
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    try {
        for (int l = 0; l <= L; l++) {
            const bool fused = ks_fused && key.fbuf && l > 0;
            float best = 0.0f;
            bool have = false;
            for (int ci = 0; ci < 4; ci++) {
                const int cfg = cands[ci];
                if (!fused && cfg != 0) continue;
                ks_tune[std::make_pair(l, nb)] = cfg;
                std::vector<float> ms;
                for (int r = 0; r <= reps; r++) {
                    HIP_CHECK(hipEventRecord(e0, st));
                    Buf acc = keyswitch_acc(d->p, (long)N, (long)(l + 1) * N, l, nb, key);
                    HIP_CHECK(hipEventRecord(e1, st));
                    HIP_CHECK(hipEventSynchronize(e1));
                    float t = 0.0f;
                    HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
                    if (r > 0) ms.push_back(t);
                }
                std::sort(ms.begin(), ms.end());
                const float med = ms[ms.size() / 2];
                if (!have || med < best) {
                    best = med;
                    chosen[l] = cfg;
                    have = true;
                }
            }
            ks_tune[std::make_pair(l, nb)] = chosen[l];
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return chosen;
}

// ModDown of a relinearisation's accumulators followed by the rescale by q_l,
// in the residues of moddown_into and rescale_affine but with one forward
// transform per limb instead of two: limb l of the sum goes first (ModDown of
// that limb alone, then to coefficient form); every other limb's transform
// then takes ModDown's conversion plus P (mod q_i) times the rescale's input
// word, and its tail forms (base + (acc - v) P^-1) k q_l^-1 (the transform is
// linear, so this is (c_i - NTT(r_i)) k q_l^-1 with c = base + ModDown(acc))
void Ctx::moddown_rescale_into(const Buf &acc, int l, int nb, const u64 *base, long base_ls, long base_es, long k,
                               const double *cadd, Ct &out)
{
    const int nq = l + 1, next = nq + alpha, np = 2 * nb;
    n_rescale++;
    Buf yP = alloc((size_t)np * alpha * N);
    launch_intt_from(T, PolySet{yP->p, (long)N, (long)alpha * N, alpha, np}, LimbMap{0, L1},
                     acc->p + (size_t)nq * N, (long)N, (long)next * N, 0, md_tab->p, md_tab->p + alpha, st, &timer);
    // limb l: ModDown of that limb alone (prime q_l through the limb map's offset,
    // every table and operand pointer moved to limb l), then coefficient form
    Buf cl = alloc((size_t)np * N), wl = alloc((size_t)np * N), last = alloc((size_t)np * N);
    OutModdownArgs oa{acc->p + (size_t)l * N, (long)N, (long)next * N, base + (size_t)l * base_ls, base_ls, base_es,
                      (long)N, 3, 0, cl->p, 0, (long)N, pinv->p + l, pinv->p + L + 1 + l};
    oa.pinvf = (const TwF *)(pinv->p + 2 * (L + 1)) + l;
    launch_moddown(T, wl->p, 1, alpha, np, LimbMap{1, L1, l}, yP->p, md_tab->p + 2 * alpha + l, L + 1, oa, st,
                   &timer);
    launch_intt_from(T, PolySet{last->p, (long)N, (long)N, 1, np}, LimbMap{1, L1, l}, cl->p, (long)N, (long)N, 0,
                     nullptr, nullptr, st, &timer);
    wl.reset();
    // limbs 0..l-1
    Buf tmp = alloc((size_t)l * np * N);
    const Buf &inv = rescale_table(l, k);
    OutModdownRescaleArgs ra{acc->p, (long)N, (long)next * N, base, base_ls, base_es, (long)N, out.d(),
                             2l * N * nb, (long)N, pinv->p, pinv->p + L + 1,
                             (const TwF *)(pinv->p + 2 * (L + 1)), inv->p, inv->p + l,
                             (const TwF *)(inv->p + 2 * l), cadd ? rescale_addend(l, k, *cadd) : nullptr};
    launch_moddown_rescale(T, tmp->p, l, alpha, np, yP->p, md_tab->p + 2 * alpha, L + 1, last->p, q[l],
                           pmod->p, pmod->p + L + 1, (const TwF *)(pmod->p + 2 * (L + 1)), ra, L1, st, &timer);
    n_launch += 8;
}

Tensor Ctx::tensor(const Ct &a, const Ct &b)
{
    if (a.level != b.level || a.nb != b.nb) throw HeError(-1, "tensor: level mismatch");
    Tensor t;
    t.level = a.level;
    t.nb = a.nb;
    t.buf = alloc((size_t)(a.level + 1) * 3 * N * a.nb);
    launch_tensor(d_pc, PolySet{t.buf->p, 3l * N * a.nb, 3l * N, a.level + 1, a.nb}, c0set(a), c0set(b),
                  lmap(a.level + 1), N, false, st);
    n_launch++;
    return t;
}

void Ctx::tensor_acc(Tensor &t, const Ct &a, const Ct &b)
{
    if (a.level != b.level || a.level != t.level || a.nb != t.nb || b.nb != t.nb)
        throw HeError(-1, "tensor: level mismatch");
    launch_tensor(d_pc, PolySet{t.buf->p, 3l * N * a.nb, 3l * N, a.level + 1, a.nb}, c0set(a), c0set(b),
                  lmap(a.level + 1), N, true, st);
    n_launch++;
}

Ct Ctx::relin_rescale(const Tensor &t, const Keys &k, long mul, const double *cadd)
{
    const u64 *tb = t.buf->p;
    const long ls = 3l * N * t.nb, es = 3l * N;
    if (!k.has_relin) throw HeError(-5, "no relinearisation key");
    if (t.level >= 1) {
        Buf acc = keyswitch_acc(tb + 2 * (size_t)N, ls, es, t.level, t.nb, k.relin);
        Ct o = new_ct(t.level - 1, t.nb);
        moddown_rescale_into(acc, t.level, t.nb, tb, ls, es, mul, cadd, o);
        return o;
    }
    Ct c = new_ct(t.level, t.nb);
    keyswitch(tb + 2 * (size_t)N, ls, es, t.level, t.nb, k.relin, 0, tb, ls, es, 3, c);
    return rescale_affine(c, mul, cadd);
}

Ct Ctx::mul(const Ct &a, const Ct &b, const Keys &k) { return relin_rescale(tensor(a, b), k); }

Ct Ctx::mul_affine(const Ct &a, const Ct &b, const Keys &keys, long k, const double *c)
{
    return relin_rescale(tensor(a, b), keys, k, c);
}

std::vector<Ct> Ctx::rotate_many(const Ct &a, const std::vector<long> &steps, const Keys &k)
{
    std::vector<Ct> out;
    bool need = false;
    for (long s : steps) need |= galois_elt(s) != 1;
    const long ls = 2l * N * a.nb, es = 2l * N;
    ModUp m;
    if (need) m = modup(a.d() + N, ls, es, a.level, a.nb);
    for (long s : steps) {
        u64 g = galois_elt(s);
        if (g == 1) {
            out.push_back(a);
            continue;
        }
        auto it = k.galois.find(g);
        if (it == k.galois.end()) throw HeError(-5, "no Galois key for rotation step " + std::to_string(s));
        Ct o = new_ct(a.level, a.nb);
        keyswitch_from(m, it->second, g, a.d(), ls, es, 1, o);
        out.push_back(o);
    }
    return out;
}

Ct Ctx::rotate_add(const Ct &a, long step, const Ct &addend, const Keys &k)
{
    u64 g = galois_elt(step);
    if (g == 1) return add(addend, a);
    auto it = k.galois.find(g);
    if (it == k.galois.end()) throw HeError(-5, "no Galois key for rotation step " + std::to_string(step));
    Ct o = new_ct(a.level, a.nb);
    const long ls = 2l * N * a.nb, es = 2l * N;
    keyswitch(a.d() + N, ls, es, a.level, a.nb, it->second, g, a.d(), ls, es, 1, o, &addend);
    return o;
}

Ct Ctx::rotate_sum(const std::vector<std::pair<const Ct *, long>> &items, const Keys &k)
{
    if (items.empty()) throw HeError(-1, "rotate_sum: no terms");
    const int l = items[0].first->level, nb = items[0].first->nb;
    for (auto &it : items)
        if (it.first->level != l || it.first->nb != nb) throw HeError(-1, "rotate_sum: operand shapes differ");
    const int nq = l + 1, next = nq + alpha;
    const long ls = 2l * N * nb, es = 2l * N;
    // the unrotated terms, summed
    Ct u;
    bool have_u = false;
    for (auto &it : items) {
        if (galois_elt(it.second) != 1) continue;
        u = have_u ? add(u, *it.first) : *it.first;
        have_u = true;
    }
    // the rotated terms: sigma_g of each accumulator into A (Q_l u P), with
    // P sigma_g(c_0) added to component 0's Q limbs (ModDown's division by P
    // makes it sigma_g(c_0), exactly, as in a single rotation's tail)
    Buf A;
    for (auto &it : items) {
        const u64 g = galois_elt(it.second);
        if (g == 1) continue;
        auto kit = k.galois.find(g);
        if (kit == k.galois.end()) throw HeError(-5, "no Galois key for rotation step " + std::to_string(it.second));
        const Ct &x = *it.first;
        Buf acc = keyswitch_acc(x.d() + N, ls, es, l, nb, kit->second);
        const bool first = !A;
        if (first) A = alloc((size_t)nb * 2 * next * N);
        launch_automorph_acc(d_pc, PolySet{A->p, (long)N, (long)next * N, next, 2 * nb},
                             PolySet{acc->p, (long)N, (long)next * N, next, 2 * nb}, c0set(x), pmod->p,
                             pmod->p + L + 1, g, logN, lmap(nq), nq, !first, st);
        n_launch++;
    }
    if (!A) return u;
    // ModDown of the summed accumulators, the unrotated sum as the addend
    Ct o = new_ct(l, nb);
    moddown_into(A, l, nb, 1, nullptr, 0, 0, 0, o, have_u ? &u : nullptr);
    return o;
}

Ct Ctx::rotate(const Ct &a, long step, const Keys &k)
{
    u64 g = galois_elt(step);
    if (g == 1) return a;
    auto it = k.galois.find(g);
    if (it == k.galois.end()) throw HeError(-5, "no Galois key for rotation step " + std::to_string(step));
    Ct o = new_ct(a.level, a.nb);
    const long ls = 2l * N * a.nb, es = 2l * N;
    keyswitch(a.d() + N, ls, es, a.level, a.nb, it->second, g, a.d(), ls, es, 1, o);
    return o;
}

// ------------------------------------------------------------- plaintexts
Buf Ctx::encode_ntt(const double *z, size_t n, double scale, int nl, bool montgomery)
{
    std::vector<u64> host((size_t)nl * N);
    encode_rns(z, n, scale, logN, mods.data(), nl, host.data());
    Buf b = alloc(host.size());
    upload(b->p, host.data(), host.size());
    PolySet ps{b->p, (long)N, 0, nl, 1};
    ntt(ps, lmap(nl), false);
    if (montgomery) {
        launch_to_montgomery(d_pc, b->p, (long)N, nl, lmap(nl), N, 1, 0, st);
        n_launch++;
    }
    return b;
}

Pt Ctx::const_pt(double c, double scale, int nl)
{
    u64 kc, ks;
    std::memcpy(&kc, &c, 8);
    std::memcpy(&ks, &scale, 8);
    auto key = std::make_pair(kc ^ 0x9e3779b97f4a7c15ull, ks);
    Pt p;
    p.is_const = true;
    p.nl = L + 1;
    auto it = const_cache.find(key);
    if (it != const_cache.end()) {
        p.buf = it->second;
        p.plain = const_plain_cache.at(key);
        return p;
    }
    std::vector<u64> v(L + 1), w(4 * (size_t)(L + 1));
    encode_const_rns(c, scale, q.data(), L + 1, v.data());
    for (int i = 0; i <= L; i++) {
        w[i] = v[i];
        w[L + 1 + i] = shoup_of(v[i], q[i]);
        w[2 * (L + 1) + i] = hmul(v[i], pc[i].ninv, q[i]);
        w[3 * (L + 1) + i] = shoup_of(w[2 * (L + 1) + i], q[i]);
        v[i] = (u64)(((u128)v[i] << 64) % q[i]);
    }
    Buf b = alloc(v.size()), bp = alloc(w.size());
    upload(b->p, v.data(), v.size());
    upload(bp->p, w.data(), w.size());
    const_cache.emplace(key, b);
    const_plain_cache.emplace(key, bp);
    p.buf = b;
    p.plain = bp;
    return p;
}

Pt Ctx::vec_pt(const double *z, size_t n, double scale, int nl)
{
    Pt p;
    p.is_const = false;
    p.nl = nl;
    p.buf = encode_ntt(z, n, scale, nl, true);
    return p;
}

std::vector<Pt> Ctx::vec_pts(const std::vector<const std::vector<double> *> &zs, double scale, int nl,
                             const std::vector<const std::vector<double> *> *ims)
{
    if (ims && ims->size() != zs.size()) throw HeError(-1, "vec_pts: real and imaginary parts differ in count");
    const size_t n = zs.size();
    std::vector<std::vector<u64>> host(n);
    std::vector<std::thread> th;
    std::exception_ptr err;
    std::mutex mu;
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (unsigned tid = 0; tid < nth; tid++)
        th.emplace_back([&, tid]() {
            try {
                for (size_t i = tid; i < n; i += nth) {
                    host[i].resize((size_t)nl * N);
                    const double *im = nullptr;
                    if (ims) {
                        if ((*ims)[i]->size() != zs[i]->size()) throw HeError(-1, "vec_pts: part sizes differ");
                        im = (*ims)[i]->data();
                    }
                    encode_rns_c(zs[i]->data(), im, zs[i]->size(), scale, logN, mods.data(), nl, host[i].data());
                }
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                err = std::current_exception();
            }
        });
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
    std::vector<Pt> out(n);
    for (size_t i = 0; i < n; i++) {
        Buf b = alloc(host[i].size());
        upload(b->p, host[i].data(), host[i].size());
        PolySet ps{b->p, (long)N, 0, nl, 1};
        ntt(ps, lmap(nl), false);
        launch_to_montgomery(d_pc, b->p, (long)N, nl, lmap(nl), N, 1, 0, st);
        n_launch++;
        out[i].is_const = false;
        out[i].nl = nl;
        out[i].buf = b;
    }
    return out;
}

// sum_i ct_i * z_i landing at level t: every ct_i is read on limbs 0..t+1
// (mod-drop), multiplied by its plaintext (encoded by the caller at
// S[t] q_{t+1} / S[level_i]), summed with one REDC per coefficient, and
// rescaled once.
Ct Ctx::lincomb(const std::vector<std::pair<const Ct *, const Pt *>> &terms, int t, const double *c)
{
    if (terms.empty()) throw HeError(-1, "lincomb: no terms");
    if (t < 0) throw HeError(-3, "lincomb: no level left");
    if (terms.size() == 1 && terms[0].second->is_const && terms[0].second->plain)
        return rescale_const_mul(*terms[0].first, *terms[0].second, t, c);
    const int nl = t + 2, nb = terms[0].first->nb;
    Ct acc = new_ct(t + 1, nb);
    const int CH = 15;
    bool first = true;
    for (size_t s0 = 0; s0 < terms.size(); s0 += CH) {
        size_t s1 = std::min(terms.size(), s0 + CH);
        std::vector<const u64 *> ab, pb;
        for (size_t i = s0; i < s1; i++) {
            if (terms[i].first->level < t + 1) throw HeError(-3, "lincomb: operand below target level");
            if (terms[i].first->nb != nb) throw HeError(-1, "lincomb: batch mismatch");
            if (terms[i].second->nl < nl) throw HeError(-1, "lincomb: plaintext has too few limbs");
            ab.push_back(terms[i].first->d());
            const u64 *pp = terms[i].second->buf->p;
            if (terms[i].second->is_const) pp = (const u64 *)((uintptr_t)pp | 1);
            pb.push_back(pp);
        }
        if (first) {
            launch_lincomb(d_pc, ctset(acc), ab.data(), 2l * N * nb, (long)N, pb.data(), (long)N, (int)ab.size(),
                           lmap(nl), N, st);
            first = false;
        } else {
            Ct part = new_ct(t + 1, nb);
            launch_lincomb(d_pc, ctset(part), ab.data(), 2l * N * nb, (long)N, pb.data(), (long)N, (int)ab.size(),
                           lmap(nl), N, st);
            launch_addsub(d_pc, ctset(acc), ctset(acc), ctset(part), lmap(nl), 0, N, st);
            n_launch++;
        }
        n_launch++;
    }
    return rescale_affine(acc, 1, c);
}

Ct Ctx::level_down(const Ct &a, int t)
{
    if (a.level == t) return a;
    if (a.level < t) throw HeError(-3, "level_down: target above operand");
    if (t < 0) throw HeError(-3, "level_down: no level left");
    Pt one = const_pt(1.0, S[t] * (double)q[t + 1] / S[a.level], t + 2);
    return lincomb({{&a, &one}}, t);
}

// ----------------------------------------------------------- batches
Ct Ctx::pack(const std::vector<const Ct *> &cts)
{
    if (cts.empty()) throw HeError(-1, "pack: empty batch");
    const int l = cts[0]->level, nb = (int)cts.size();
    Ct o = new_ct(l, nb);
    for (int e = 0; e < nb; e++) {
        if (cts[e]->level != l || cts[e]->nb != 1) throw HeError(-1, "pack: ciphertexts at different levels");
        launch_copy(PolySet{o.d() + (size_t)e * 2 * N, 2l * N * nb, (long)N, l + 1, 2}, ctset(*cts[e]), N, st);
        n_launch++;
    }
    return o;
}

Ct Ctx::unpack(const Ct &b, int e)
{
    Ct o = new_ct(b.level, 1);
    launch_copy(ctset(o), PolySet{b.d() + (size_t)e * 2 * N, 2l * N * b.nb, (long)N, b.level + 1, 2}, N, st);
    n_launch++;
    return o;
}

// ------------------------------------------------------------------- client
void Ctx::gen_switch_key(const u64 *s_ntt, u64 seed, u32 key_id, const u64 *sp_ntt, SwitchKey &out)
{
    const int ktot = L + 1 + alpha, dn = dnum_top();
    out.buf = alloc((size_t)dn * 2 * ktot * N);
    std::vector<u64> a((size_t)ktot * N), e((size_t)ktot * N), pf(ktot);
    std::vector<int64_t> es(N);
    Buf de = alloc((size_t)ktot * N), dpf = alloc(ktot);
    u64 P_mod[64];
    for (int t = 0; t < ktot; t++) {
        u64 m = mods[t], P = 1;
        for (u64 pj : p) P = hmul(P, pj % m, m);
        P_mod[t] = P;
    }
    for (int j = 0; j < dn; j++) {
        // uniform a_j per limb in parallel host threads (independent streams)
        std::vector<std::thread> th;
        int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (int tid = 0; tid < nth; tid++)
            th.emplace_back([&, tid]() {
                for (int t = tid; t < ktot; t += nth)
                    sample_uniform(seed, 2, key_id, ((u32)j << 16) | (u32)t, mods[t], N, &a[(size_t)t * N]);
            });
        for (auto &x : th) x.join();
        sample_gauss(seed, 3, key_id, (u32)j << 16, sigma, N, es.data());
        for (int t = 0; t < ktot; t++) {
            u64 m = mods[t];
            for (int n = 0; n < N; n++) {
                int64_t v = es[n];
                e[(size_t)t * N + n] = v < 0 ? m - (u64)(-v) : (u64)v;
            }
            pf[t] = (t <= L && t >= j * w && t < j * w + w) ? P_mod[t] : 0;
        }
        u64 *kb = out.buf->p + (size_t)j * 2 * ktot * N;
        u64 *ka = kb + (size_t)ktot * N;
        upload(ka, a.data(), a.size());
        upload(de->p, e.data(), e.size());
        upload(dpf->p, pf.data(), pf.size());
        LimbMap lm = lmap(L + 1);
        ntt(PolySet{ka, (long)N, 0, ktot, 1}, lm, false);
        ntt(PolySet{de->p, (long)N, 0, ktot, 1}, lm, false);
        launch_keygen_b(d_pc, kb, ka, s_ntt, de->p, sp_ntt, dpf->p, ktot, N, st);
        n_launch++;
    }
    sync();
}

// the double copy of a key's FP64-prime limbs read by the fused ModUp products
// (from the key as stored, i.e. after a Galois key's permutation)
void Ctx::key_fp(SwitchKey &k)
{
    if (!ks_fused) return;
    const int ktot = L + 1 + alpha, dn = dnum_top();
    k.fbuf = alloc((size_t)dn * 2 * ktot * N);
    launch_key_fp(d_pc, k.buf->p, k.fbuf->p, dn * 2 * ktot, ktot, N, st);
    n_launch++;
}

Buf Ctx::secret_ntt(const SecretKey &sk, int nl)
{
    const int ktot = nl;
    std::vector<u64> sr((size_t)ktot * N);
    for (int t = 0; t < ktot; t++)
        for (int n = 0; n < N; n++) {
            int64_t v = sk.s[n];
            sr[(size_t)t * N + n] = v < 0 ? mods[t] - 1 : (u64)v;
        }
    Buf b = alloc(sr.size());
    upload(b->p, sr.data(), sr.size());
    std::fill(sr.begin(), sr.end(), 0);
    ntt(PolySet{b->p, (long)N, 0, ktot, 1}, lmap(std::min(nl, L + 1)), false);
    return b;
}

void Ctx::wipe(const Buf &b)
{
    HIP_CHECK(hipMemsetAsync(b->p, 0, b->words * sizeof(u64), st));
    sync();
}

// Galois keys are stored as sigma_g^-1(key), so the inner product needs no permutation
static void store_galois(Ctx &c, SwitchKey &gk, u64 g)
{
    const size_t words = (size_t)c.dnum_top() * 2 * (c.L + 1 + c.alpha) * c.N;
    Buf perm = c.alloc(words);
    launch_automorph(PolySet{perm->p, (long)c.N, 0, (int)(words / c.N), 1},
                     PolySet{gk.buf->p, (long)c.N, 0, (int)(words / c.N), 1}, hinv(g, 2ull * c.N), c.logN, c.st);
    c.n_launch++;
    gk.buf = perm;
    c.key_fp(gk);
}

void Ctx::keygen(u64 seed, const std::vector<long> &steps, SecretKey *&sk_out, Keys *&ek_out)
{
    const int ktot = L + 1 + alpha;
    std::unique_ptr<SecretKey> sk(new SecretKey());
    sk->ctx = this;
    sk->s.resize(N);
    if (hamming > 0)
        sample_sparse_ternary(seed, 1, 0, 0, N, hamming, sk->s.data());
    else
        sample_ternary(seed, 1, 0, 0, N, sk->s.data());
    std::unique_ptr<Keys> k(new Keys());
    k->ctx = this;
    Buf s_ntt = secret_ntt(*sk, ktot);
    LimbMap lm = lmap(L + 1);
    PolySet sset{s_ntt->p, (long)N, 0, ktot, 1};
    // relinearisation key: s' = s^2 (pointwise in the NTT domain)
    Buf s2 = alloc((size_t)ktot * N);
    launch_pmul(d_pc, PolySet{s2->p, (long)N, 0, ktot, 1}, sset, sset, lm, N, st);
    n_launch++;
    gen_switch_key(s_ntt->p, seed, 0, s2->p, k->relin);
    k->has_relin = true;
    key_fp(k->relin);
    // Galois keys: s' = sigma_g(s), a permutation of NTT slots
    Buf sg = alloc((size_t)ktot * N);
    for (long step : steps) {
        u64 g = galois_elt(step);
        if (g == 1 || k->galois.count(g)) continue;
        launch_automorph(PolySet{sg->p, (long)N, 0, ktot, 1}, sset, g, logN, st);
        n_launch++;
        SwitchKey &gk = k->galois[g];
        gen_switch_key(s_ntt->p, seed, (u32)g, sg->p, gk);
        store_galois(*this, gk, g);
    }
    wipe(s_ntt);
    wipe(s2);
    wipe(sg);
    sk_out = sk.release();
    ek_out = k.release();
}

Keys *Ctx::import_keys(const std::vector<u32> &ids, const std::vector<const u64 *> &data)
{
    const int ktot = L + 1 + alpha, dn = dnum_top();
    const size_t words = (size_t)dn * 2 * ktot * N;
    std::unique_ptr<Keys> k(new Keys());
    k->ctx = this;
    for (size_t i = 0; i < ids.size(); i++) {
        const u32 id = ids[i];
        if (id != 0 && ((id & 1) == 0 || id >= 2u * (u32)N))
            throw HeError(-1, "key id " + std::to_string(id) + " is not a Galois element");
        if (id == 0 ? k->has_relin : k->galois.count(id) != 0) throw HeError(-1, "repeated key id");
        const u64 *src = data[i];
        if (!src) throw HeError(-1, "null key data");
        for (size_t r = 0; r < (size_t)dn * 2 * ktot; r++) {
            const u64 m = mods[r % ktot];
            for (int n = 0; n < N; n++)
                if (src[r * N + n] >= m) throw HeError(-1, "key residue not reduced");
        }
        SwitchKey sw;
        sw.buf = alloc(words);
        upload(sw.buf->p, src, words);
        // coefficient form -> NTT form -> Montgomery form, as keygen leaves them
        PolySet ps{sw.buf->p, (long)N, (long)ktot * N, ktot, dn * 2};
        LimbMap lm = lmap(L + 1);
        ntt(ps, lm, false);
        launch_to_montgomery(d_pc, sw.buf->p, (long)N, ktot, lm, N, dn * 2, (long)ktot * N, st);
        n_launch++;
        if (id == 0) {
            k->relin = sw;
            k->has_relin = true;
            key_fp(k->relin);
        } else {
            SwitchKey &gk = k->galois[id];
            gk = sw;
            store_galois(*this, gk, id);
        }
    }
    sync();
    return k.release();
}

void Ctx::export_key(const Keys &k, u32 key_id, int digit, u64 *out)
{
    const int ktot = L + 1 + alpha;
    if (digit < 0 || digit >= dnum_top()) throw HeError(-1, "digit out of range");
    const SwitchKey *sk = nullptr;
    if (key_id == 0) {
        if (!k.has_relin) throw HeError(-5, "no relinearisation key");
        sk = &k.relin;
    } else {
        auto it = k.galois.find(key_id);
        if (it == k.galois.end()) throw HeError(-5, "no such key");
        sk = &it->second;
    }
    Buf tmp = alloc((size_t)2 * ktot * N);
    const u64 *src = sk->buf->p + (size_t)digit * 2 * ktot * N;
    if (key_id == 0) {
        HIP_CHECK(hipMemcpyAsync(tmp->p, src, (size_t)2 * ktot * N * 8, hipMemcpyDeviceToDevice, st));
    } else {
        // Galois keys are stored permuted by sigma^-1: undo it
        launch_automorph(PolySet{tmp->p, (long)N, 0, 2 * ktot, 1}, PolySet{(u64 *)src, (long)N, 0, 2 * ktot, 1},
                         key_id, logN, st);
    }
    // leave Montgomery form: multiply by 2^-64 mod q
    std::vector<u64> inv(2 * ktot);
    for (int t = 0; t < ktot; t++) {
        u64 m = mods[t];
        inv[t] = hinv(pc[t].r1, m);
        inv[ktot + t] = shoup_of(inv[t], m);
    }
    Buf dinv = alloc(inv.size());
    upload(dinv->p, inv.data(), inv.size());
    LimbMap lm = lmap(L + 1);
    PolySet ps{tmp->p, (long)N, (long)ktot * N, ktot, 2};
    launch_mul_scalar(d_pc, ps, ps, dinv->p, dinv->p + ktot, lm, N, st);
    ntt(ps, lm, true);
    download(out, tmp->p, (size_t)2 * ktot * N);
}

Ct Ctx::encrypt(const SecretKey &sk, const double *x, size_t n, u64 seed)
{
    const int nl = top + 1;
    if (n > (size_t)N / 2) throw HeError(-4, "encrypt: more values than slots");
    std::vector<u64> em((size_t)nl * N), a((size_t)nl * N);
    encode_rns(x, n, S[top], logN, q.data(), nl, em.data());
    std::vector<int64_t> e(N);
    sample_gauss(seed, 5, 0, 0, sigma, N, e.data());
    for (int t = 0; t < nl; t++) {
        u64 m = q[t];
        for (int i = 0; i < N; i++) {
            int64_t v = e[i];
            u64 r = v < 0 ? m - (u64)(-v) : (u64)v;
            u64 &dst = em[(size_t)t * N + i];
            dst = dst + r >= m ? dst + r - m : dst + r;
        }
        sample_uniform(seed, 4, 0, (u32)t, m, N, &a[(size_t)t * N]);
    }
    Buf da = alloc(a.size()), dem = alloc(em.size());
    upload(da->p, a.data(), a.size());
    upload(dem->p, em.data(), em.size());
    LimbMap lm = lmap(nl);
    ntt(PolySet{da->p, (long)N, 0, nl, 1}, lm, false);
    ntt(PolySet{dem->p, (long)N, 0, nl, 1}, lm, false);
    Ct c = new_ct(top);
    Buf s_ntt = secret_ntt(sk, nl);
    launch_copy(PolySet{c.d() + N, 2l * N, 0, nl, 1}, PolySet{da->p, (long)N, 0, nl, 1}, N, st);
    launch_encrypt(d_pc, c.d(), c.d() + N, s_ntt->p, dem->p, 2l * N, nl, N, st);
    n_launch += 2;
    wipe(s_ntt);
    return c;
}

void Ctx::decrypt(const SecretKey &sk, const Ct &c, double *y, size_t n)
{
    Buf m = alloc(N);
    Buf s_ntt = secret_ntt(sk, 1);
    launch_decrypt0(d_pc, m->p, c.d(), c.d() + N, s_ntt->p, N, st);
    wipe(s_ntt);
    ntt(PolySet{m->p, (long)N, 0, 1, 1}, lmap(1), true);
    std::vector<u64> h(N);
    download(h.data(), m->p, N);
    decode_limb(h.data(), q[0], S[c.level], logN, n, y);
}

}  // namespace hk
