// Device-resident RNS-CKKS operations (Preliminaries, Homomorphic Encryption:
// add, subtract, multiply, rotate), orchestrated on one HIP stream.
#include "ckks.hpp"

#include <algorithm>
#include <cstring>
#include <thread>

namespace hk {

// ------------------------------------------------------------------- memory
void *Pool::get(size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.find(bytes);
    void *p = nullptr;
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
    bytes = (bytes + 255) & ~(size_t)255;
    live -= bytes;
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
         hipStream_t stream)
    : logN(logN_), N(1 << logN_), L(L_), alpha(alpha_), w(w_), L1(L_ + 1), sigma(sigma_)
{
    make_chain(logN, base_bits, L, scale_bits, alpha, special_bits, q, p, S);
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
    }
    d_pc_buf = alloc((sizeof(PrimeConst) * np + 7) / 8);
    HIP_CHECK(hipMemcpyAsync(d_pc_buf->p, pc.data(), sizeof(PrimeConst) * np, hipMemcpyHostToDevice, st));
    d_pc = (const PrimeConst *)d_pc_buf->p;
    // twiddles: psi^brv(k) and psi^-brv(k) with Shoup companions
    std::vector<u64> tw((size_t)4 * np * N);
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
        }
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
    pinv = alloc(pv.size());
    upload(pinv->p, pv.data(), pv.size());
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
    bconv_cache.clear();
    rescale_inv.clear();
    const_cache.clear();
    int_cache.clear();
    pinv.reset();
    tw_buf.reset();
    d_pc_buf.reset();
    pool.trim();
    if (own_stream && st) (void)hipStreamDestroy(st);
}

u64 Ctx::galois_elt(long step) const
{
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
    return PolySet{c.d(), 2l * N, (long)N, nl < 0 ? c.level + 1 : nl, 2};
}

// ------------------------------------------------------------ simple ct ops
Ct Ctx::new_ct(int level)
{
    Ct c;
    c.level = level;
    c.buf = alloc((size_t)(level + 1) * 2 * N);
    return c;
}

Ct Ctx::add(const Ct &a, const Ct &b)
{
    if (a.level != b.level) throw HeError(-1, "add: level mismatch");
    Ct o = new_ct(a.level);
    launch_addsub(d_pc, ctset(o), ctset(a), ctset(b), lmap(a.level + 1), 0, N, st);
    n_launch++;
    return o;
}

Ct Ctx::sub(const Ct &a, const Ct &b)
{
    if (a.level != b.level) throw HeError(-1, "sub: level mismatch");
    Ct o = new_ct(a.level);
    launch_addsub(d_pc, ctset(o), ctset(a), ctset(b), lmap(a.level + 1), 1, N, st);
    n_launch++;
    return o;
}

Ct Ctx::mul_int(const Ct &a, long k)
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
    Ct o = new_ct(a.level);
    launch_mul_scalar(d_pc, ctset(o), ctset(a), it->second->p, it->second->p + L + 1, lmap(a.level + 1), N, st);
    n_launch++;
    return o;
}

Ct Ctx::add_const(const Ct &a, double c)
{
    double sc = S[a.level];
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
    Ct o = new_ct(a.level);
    launch_copy(ctset(o), ctset(a), N, st);
    launch_add_const(d_pc, ctset(o), it->second->p, lmap(a.level + 1), N, st);
    n_launch += 2;
    return o;
}

Ct Ctx::add_plain(const Ct &a, const Buf &pt)
{
    Ct o = new_ct(a.level);
    launch_copy(ctset(o), ctset(a), N, st);
    PolySet o0 = ctset(o);
    o0.npoly = 1;
    PolySet p0{pt->p, (long)N, 0, a.level + 1, 1};
    launch_addsub(d_pc, o0, o0, p0, lmap(a.level + 1), 0, N, st);
    n_launch += 2;
    return o;
}

Ct Ctx::mod_drop(const Ct &a, int l) const
{
    if (l > a.level || l < 0) throw HeError(-1, "mod_drop: bad level");
    Ct o = a;
    o.level = l;
    return o;
}

// ------------------------------------------------------------------ rescale
const Buf &Ctx::rescale_table(int l)
{
    auto it = rescale_inv.find(l);
    if (it != rescale_inv.end()) return it->second;
    std::vector<u64> v(2 * l);
    for (int i = 0; i < l; i++) {
        v[i] = hinv(q[l] % q[i], q[i]);
        v[l + i] = shoup_of(v[i], q[i]);
    }
    Buf b = alloc(std::max<size_t>(v.size(), 1));
    if (l) upload(b->p, v.data(), v.size());
    return rescale_inv.emplace(l, b).first->second;
}

Ct Ctx::rescale(const Ct &a)
{
    int l = a.level;
    if (l < 1) throw HeError(-3, "rescale: no level left");
    n_rescale++;
    // limb l of both polynomials to coefficient form
    Buf last = alloc(2 * (size_t)N);
    PolySet lastset{last->p, 2l * N, (long)N, 1, 2};
    PolySet src{a.d() + (size_t)l * 2 * N, 2l * N, (long)N, 1, 2};
    launch_copy(lastset, src, N, st);
    PolySet lastview{last->p - (size_t)l * 2 * N, 2l * N, (long)N, l + 1, 2};
    ntt(lastview, lmap(l + 1), true, 0, l);
    Buf tmp = alloc((size_t)l * 2 * N);
    PolySet tset{tmp->p, 2l * N, (long)N, l, 2};
    launch_rescale_prep(d_pc, tset, lastset, l, N, st);
    ntt(tset, lmap(l), false);
    Ct o = new_ct(l - 1);
    const Buf &inv = rescale_table(l);
    launch_rescale_fin(d_pc, ctset(o), ctset(a, l), tset, inv->p, inv->p + l, N, st);
    n_launch += 3;
    return o;
}

// --------------------------------------------------------- basis conversion
static BconvDev make_plan(Ctx &c, const std::vector<int> &sp, const std::vector<int> &dp,
                          const std::vector<int> &dl)
{
    int ns = (int)sp.size(), nd = (int)dp.size();
    if (ns > 8) throw HeError(-1, "basis conversion from more than 8 limbs is not supported");
    std::vector<u64> invhat(ns), invhatp(ns), hatm((size_t)ns * nd);
    for (int j = 0; j < ns; j++) {
        u64 qj = c.mods[sp[j]];
        u64 h = 1;
        for (int k = 0; k < ns; k++)
            if (k != j) h = hmul(h, c.mods[sp[k]] % qj, qj);
        invhat[j] = hinv(h, qj);
        invhatp[j] = shoup_of(invhat[j], qj);
        for (int t = 0; t < nd; t++) {
            u64 pt = c.mods[dp[t]];
            u64 hp = 1;
            for (int k = 0; k < ns; k++)
                if (k != j) hp = hmul(hp, c.mods[sp[k]] % pt, pt);
            hatm[(size_t)j * nd + t] = (u64)(((u128)hp << 64) % pt);  // Montgomery form
        }
    }
    size_t ints = (size_t)(ns + 2 * nd);
    size_t words = (ints + 1) / 2 + 2 * ns + (size_t)ns * nd;
    BconvDev d;
    d.store = c.alloc(words);
    std::vector<u64> host(words, 0);
    int32_t *ip = (int32_t *)host.data();
    for (int j = 0; j < ns; j++) ip[j] = sp[j];
    for (int t = 0; t < nd; t++) {
        ip[ns + t] = dp[t];
        ip[ns + nd + t] = dl[t];
    }
    size_t off = (ints + 1) / 2;
    std::memcpy(&host[off], invhat.data(), ns * 8);
    std::memcpy(&host[off + ns], invhatp.data(), ns * 8);
    std::memcpy(&host[off + 2 * ns], hatm.data(), hatm.size() * 8);
    c.upload(d.store->p, host.data(), words);
    int32_t *dip = (int32_t *)d.store->p;
    d.plan.ns = ns;
    d.plan.nd = nd;
    d.plan.src_prime = dip;
    d.plan.dst_prime = dip + ns;
    d.plan.dst_limb = dip + ns + nd;
    d.plan.invhat = d.store->p + off;
    d.plan.invhatp = d.store->p + off + ns;
    d.plan.hatm = d.store->p + off + 2 * ns;
    return d;
}

const BconvDev &Ctx::modup_plan(int l, int j)
{
    long key = ((long)1 << 40) | ((long)l << 20) | j;
    auto it = bconv_cache.find(key);
    if (it != bconv_cache.end()) return it->second;
    int nq = l + 1, lo = j * w, hi = std::min(lo + w, nq);
    std::vector<int> sp, dp, dl;
    for (int i = lo; i < hi; i++) sp.push_back(i);
    LimbMap lm = lmap(nq);
    for (int t = 0; t < nq + alpha; t++)
        if (t < lo || t >= hi) {
            dp.push_back(lm.prime(t));
            dl.push_back(t);
        }
    return bconv_cache.emplace(key, make_plan(*this, sp, dp, dl)).first->second;
}

const BconvDev &Ctx::moddown_plan(int l)
{
    long key = ((long)2 << 40) | ((long)l << 20);
    auto it = bconv_cache.find(key);
    if (it != bconv_cache.end()) return it->second;
    std::vector<int> sp, dp, dl;
    for (int i = 0; i < alpha; i++) sp.push_back(L1 + i);
    for (int i = 0; i <= l; i++) {
        dp.push_back(i);
        dl.push_back(i);
    }
    return bconv_cache.emplace(key, make_plan(*this, sp, dp, dl)).first->second;
}

// -------------------------------------------------------------- key switch
// Hybrid key switching (Han-Ki): d is split into digits of w Q limbs; each
// digit is extended to Q_l u P by fast basis conversion (ModUp), multiplied by
// the key digit and accumulated; the sum is divided by P (ModDown).  For a
// rotation the Galois automorphism acts on the extended digits inside the
// inner product, so rotations of the same ciphertext can share ModUp.
void Ctx::keyswitch(const u64 *d, long ls, int l, const SwitchKey &key, u64 galois, const u64 *base,
                    long base_ls, long base_ps, int base_mask, Ct &out)
{
    n_ks++;
    const int nq = l + 1, next = nq + alpha, nd = ndig(l), ktot = L + 1 + alpha;
    const LimbMap lm = lmap(nq);
    Buf dc = alloc((size_t)nq * N);
    PolySet dcs{dc->p, (long)N, 0, nq, 1};
    launch_copy(dcs, PolySet{(u64 *)d, ls, 0, nq, 1}, N, st);
    ntt(dcs, lm, true);
    Buf ext = alloc((size_t)nd * next * N);
    for (int j = 0; j < nd; j++) {
        int lo = j * w, hi = std::min(lo + w, nq);
        u64 *ej = ext->p + (size_t)j * next * N;
        launch_copy(PolySet{ej + (size_t)lo * N, (long)N, 0, hi - lo, 1},
                    PolySet{(u64 *)d + lo * ls, ls, 0, hi - lo, 1}, N, st);
        const BconvDev &bp = modup_plan(l, j);
        launch_bconv(d_pc, bp.plan, dc->p + (size_t)lo * N, (long)N, ej, (long)N, N, st, &timer);
        ntt(PolySet{ej, (long)N, 0, next, 1}, lm, false, lo, hi);
        n_launch += 2;
    }
    Buf acc = alloc((size_t)2 * next * N);
    launch_keyip(d_pc, acc->p, (long)next * N, ext->p, (long)next * N, key.buf->p, 2l * ktot * N,
                 (long)ktot * N, nd, next, lm, L1, galois, logN, st, &timer);
    // ModDown
    ntt(PolySet{acc->p + (size_t)nq * N, (long)N, (long)next * N, alpha, 2}, LimbMap{0, L1}, true);
    Buf conv = alloc((size_t)2 * nq * N);
    const BconvDev &dp = moddown_plan(l);
    for (int c = 0; c < 2; c++)
        launch_bconv(d_pc, dp.plan, acc->p + (size_t)c * next * N + (size_t)nq * N, (long)N,
                     conv->p + (size_t)c * nq * N, (long)N, N, st, &timer);
    ntt(PolySet{conv->p, (long)N, (long)nq * N, nq, 2}, lm, false);
    launch_moddown_fin(d_pc, ctset(out, nq), PolySet{(u64 *)base, base_ls, base_ps, nq, 2}, base_mask, galois,
                       acc->p, (long)N, (long)next * N, conv->p, (long)N, (long)nq * N, pinv->p,
                       pinv->p + L + 1, logN, st);
    n_launch += 5;
}

Tensor Ctx::tensor(const Ct &a, const Ct &b)
{
    if (a.level != b.level) throw HeError(-1, "tensor: level mismatch");
    Tensor t;
    t.level = a.level;
    t.buf = alloc((size_t)(a.level + 1) * 3 * N);
    launch_tensor(d_pc, PolySet{t.buf->p, 3l * N, (long)N, a.level + 1, 3}, ctset(a), ctset(b),
                  lmap(a.level + 1), N, false, st);
    n_launch++;
    return t;
}

void Ctx::tensor_acc(Tensor &t, const Ct &a, const Ct &b)
{
    if (a.level != b.level || a.level != t.level) throw HeError(-1, "tensor: level mismatch");
    launch_tensor(d_pc, PolySet{t.buf->p, 3l * N, (long)N, a.level + 1, 3}, ctset(a), ctset(b),
                  lmap(a.level + 1), N, true, st);
    n_launch++;
}

Ct Ctx::relin_rescale(const Tensor &t, const Keys &k)
{
    Ct c = new_ct(t.level);
    const u64 *tb = t.buf->p;
    keyswitch(tb + 2 * (size_t)N, 3l * N, t.level, k.relin, 0, tb, 3l * N, (long)N, 3, c);
    return rescale(c);
}

Ct Ctx::mul(const Ct &a, const Ct &b, const Keys &k) { return relin_rescale(tensor(a, b), k); }

Ct Ctx::rotate(const Ct &a, long step, const Keys &k)
{
    u64 g = galois_elt(step);
    if (g == 1) return a;
    auto it = k.galois.find(g);
    if (it == k.galois.end()) throw HeError(-5, "no Galois key for rotation step " + std::to_string(step));
    Ct o = new_ct(a.level);
    keyswitch(a.d() + N, 2l * N, a.level, it->second, g, a.d(), 2l * N, (long)N, 1, o);
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
        return p;
    }
    std::vector<u64> v(L + 1);
    encode_const_rns(c, scale, q.data(), L + 1, v.data());
    for (int i = 0; i <= L; i++) v[i] = (u64)(((u128)v[i] << 64) % q[i]);
    Buf b = alloc(v.size());
    upload(b->p, v.data(), v.size());
    const_cache.emplace(key, b);
    p.buf = b;
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

// sum_i ct_i * z_i landing at level t: every ct_i is read on limbs 0..t+1
// (mod-drop), multiplied by its plaintext (encoded by the caller at
// S[t] q_{t+1} / S[level_i]), summed with one REDC per coefficient, and
// rescaled once.
Ct Ctx::lincomb(const std::vector<std::pair<const Ct *, const Pt *>> &terms, int t)
{
    if (terms.empty()) throw HeError(-1, "lincomb: no terms");
    int nl = t + 2;
    Ct acc = new_ct(t + 1);
    const int CH = 15;
    bool first = true;
    for (size_t s0 = 0; s0 < terms.size(); s0 += CH) {
        size_t s1 = std::min(terms.size(), s0 + CH);
        std::vector<const u64 *> ab, pb;
        for (size_t i = s0; i < s1; i++) {
            if (terms[i].first->level < t + 1) throw HeError(-3, "lincomb: operand below target level");
            if (terms[i].second->nl < nl) throw HeError(-1, "lincomb: plaintext has too few limbs");
            ab.push_back(terms[i].first->d());
            const u64 *pp = terms[i].second->buf->p;
            if (terms[i].second->is_const) pp = (const u64 *)((uintptr_t)pp | 1);
            pb.push_back(pp);
        }
        if (first) {
            launch_lincomb(d_pc, ctset(acc), ab.data(), 2l * N, (long)N, pb.data(), (long)N, (int)ab.size(),
                           lmap(nl), N, st);
            first = false;
        } else {
            Ct part = new_ct(t + 1);
            launch_lincomb(d_pc, ctset(part), ab.data(), 2l * N, (long)N, pb.data(), (long)N, (int)ab.size(),
                           lmap(nl), N, st);
            launch_addsub(d_pc, ctset(acc), ctset(acc), ctset(part), lmap(nl), 0, N, st);
            n_launch++;
        }
        n_launch++;
    }
    return rescale(acc);
}

Ct Ctx::level_down(const Ct &a, int t)
{
    if (a.level == t) return a;
    if (a.level < t) throw HeError(-3, "level_down: target above operand");
    Pt one = const_pt(1.0, S[t] * (double)q[t + 1] / S[a.level], t + 2);
    return lincomb({{&a, &one}}, t);
}

// ------------------------------------------------------------------- client
void Ctx::gen_switch_key(Keys &k, u64 seed, u32 key_id, const u64 *sp_ntt, SwitchKey &out)
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
        launch_keygen_b(d_pc, kb, ka, k.s_ntt->p, de->p, sp_ntt, dpf->p, ktot, N, st);
        n_launch++;
    }
    sync();
}

Keys *Ctx::keygen(u64 seed, const std::vector<long> &steps)
{
    const int ktot = L + 1 + alpha;
    std::unique_ptr<Keys> k(new Keys());
    k->ctx = this;
    k->s.resize(N);
    sample_ternary(seed, 1, 0, 0, N, k->s.data());
    std::vector<u64> sr((size_t)ktot * N);
    for (int t = 0; t < ktot; t++)
        for (int n = 0; n < N; n++) {
            int64_t v = k->s[n];
            sr[(size_t)t * N + n] = v < 0 ? mods[t] - 1 : (u64)v;
        }
    k->s_ntt = alloc(sr.size());
    upload(k->s_ntt->p, sr.data(), sr.size());
    LimbMap lm = lmap(L + 1);
    PolySet sset{k->s_ntt->p, (long)N, 0, ktot, 1};
    ntt(sset, lm, false);
    // relinearisation key: s' = s^2 (pointwise in the NTT domain)
    Buf s2 = alloc(sr.size());
    launch_pmul(d_pc, PolySet{s2->p, (long)N, 0, ktot, 1}, sset, sset, lm, N, st);
    n_launch++;
    gen_switch_key(*k, seed, 0, s2->p, k->relin);
    // Galois keys: s' = sigma_g(s), a permutation of NTT slots
    Buf sg = alloc(sr.size());
    for (long step : steps) {
        u64 g = galois_elt(step);
        if (g == 1 || k->galois.count(g)) continue;
        launch_automorph(PolySet{sg->p, (long)N, 0, ktot, 1}, sset, g, logN, st);
        n_launch++;
        gen_switch_key(*k, seed, (u32)g, sg->p, k->galois[g]);
    }
    return k.release();
}

Ct Ctx::encrypt(const Keys &k, const double *x, size_t n, u64 seed)
{
    const int nl = L + 1;
    if (n > (size_t)N / 2) throw HeError(-4, "encrypt: more values than slots");
    std::vector<u64> em((size_t)nl * N), a((size_t)nl * N);
    encode_rns(x, n, S[L], logN, q.data(), nl, em.data());
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
    Ct c = new_ct(L);
    launch_copy(PolySet{c.d() + N, 2l * N, 0, nl, 1}, PolySet{da->p, (long)N, 0, nl, 1}, N, st);
    launch_encrypt(d_pc, c.d(), c.d() + N, k.s_ntt->p, dem->p, 2l * N, nl, N, st);
    n_launch += 2;
    return c;
}

void Ctx::decrypt(const Keys &k, const Ct &c, double *y, size_t n)
{
    Buf m = alloc(N);
    launch_decrypt0(d_pc, m->p, c.d(), c.d() + N, k.s_ntt->p, N, st);
    ntt(PolySet{m->p, (long)N, 0, 1, 1}, lmap(1), true);
    std::vector<u64> h(N);
    download(h.data(), m->p, N);
    decode_limb(h.data(), q[0], S[c.level], logN, n, y);
}

}  // namespace hk
