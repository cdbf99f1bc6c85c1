// extern "C" boundary of the library (declared in include/hekan.h).
#include <algorithm>
#include <cstring>

#include <functional>

#include "handles.hpp"

extern "C" {

int he_ctx_create(const he_params *p, void *hip_stream, he_ctx **out)
{
    if (!p || !out) return HE_EINVAL;
    *out = nullptr;
    he_ctx *h = new he_ctx();
    int rc = guard(h, [&]() {
        need(p->log_n >= 10 && p->log_n <= 16, "log_n must be in [10, 16]");
        need(p->levels >= 1 && p->levels + 1 + p->special_count <= 64, "levels out of range");
        need(p->scale_bits >= 20 && p->scale_bits <= 58, "scale_bits out of range");
        need(p->base_bits > p->scale_bits && p->base_bits <= 60, "base_bits out of range");
        need(p->special_bits >= 20 && p->special_bits <= 60, "special_bits out of range");
        need(p->special_count >= 1 && p->special_count <= 8, "special_count out of range");
        need(p->digit_width >= 1 && p->digit_width <= 8, "digit_width out of range");
        need((p->levels + p->digit_width) / p->digit_width <= 16, "more than 16 key-switch digits");
        need(p->sigma > 0 && p->sigma < 100, "sigma out of range");
        need(p->boot_levels >= 0 && p->boot_levels < p->levels, "boot_levels out of range");
        need(p->boot_levels == 0 || (p->boot_bits >= 20 && p->boot_bits <= 58), "boot_bits out of range");
        need(p->secret_hamming_weight >= 0 && p->secret_hamming_weight <= (1 << p->log_n),
             "secret_hamming_weight out of range");
        h->c = new Ctx(p->log_n, p->levels, p->scale_bits, p->base_bits, p->special_count, p->special_bits,
                       p->digit_width, p->sigma, (hipStream_t)hip_stream, p->integer_words != 0, p->boot_levels,
                       p->boot_bits, p->secret_hamming_weight);
    });
    if (rc != HE_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return HE_OK;
}

int he_ctx_destroy(he_ctx *ctx)
{
    if (!ctx) return HE_EINVAL;
    release(ctx);
    return HE_OK;
}

const char *he_last_error(const he_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int he_ctx_primes(const he_ctx *ctx, uint64_t *q, uint64_t *p, double *scales)
{
    if (!ctx) return HE_EINVAL;
    const Ctx &c = *ctx->c;
    if (q) std::memcpy(q, c.q.data(), c.q.size() * 8);  // same 64-bit layout
    if (p) std::memcpy(p, c.p.data(), c.p.size() * 8);
    if (scales) std::memcpy(scales, c.S.data(), c.S.size() * 8);
    return HE_OK;
}

int he_ctx_counters(const he_ctx *ctx, uint64_t *ks, uint64_t *rs, uint64_t *launches)
{
    if (!ctx) return HE_EINVAL;
    if (ks) *ks = ctx->c->n_ks;
    if (rs) *rs = ctx->c->n_rescale;
    if (launches) *launches = ctx->c->n_launch;
    return HE_OK;
}

int he_ctx_sync(he_ctx *ctx)
{
    if (!ctx) return HE_EINVAL;
    return guard(ctx, [&]() { ctx->c->sync(); });
}

int he_ctx_profile(he_ctx *ctx, int32_t kernel)
{
    if (!ctx || kernel < -1 || kernel >= KID_COUNT) return HE_EINVAL;
    return guard(ctx, [&]() { ctx->c->profile(kernel); });
}

int he_ctx_autotune(he_ctx *ctx, const he_eval_keys *k, int32_t batch, int32_t reps, int32_t *choice, size_t cap,
                    size_t *n)
{
    if (!ctx || !k || !n || batch < 1 || reps < 1 || (cap && !choice)) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        if (!k->k->has_relin) throw HeError(HE_EKEY, "no relinearisation key");
        const std::vector<int> c = ctx->c->autotune_keyswitch(k->k->relin, batch, reps);
        *n = c.size();
        for (size_t i = 0; i < c.size() && i < cap; i++) choice[i] = c[i];
    });
}

int he_ctx_bench_keyswitch(he_ctx *ctx, const he_eval_keys *k, int32_t step, int32_t level, int32_t batch,
                           int32_t reps, double *ms)
{
    if (!ctx || !k || !ms || batch < 1 || reps < 1) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        Ctx &c = *ctx->c;
        need(level >= 0 && level <= c.L, "level out of range");
        if (step == 0) {
            if (level < 1) throw HeError(HE_EDEPTH, "a relinearised product needs level >= 1");
            if (!k->k->has_relin) throw HeError(HE_EKEY, "no relinearisation key");
        } else if (!k->k->galois.count(c.galois_elt(step))) {
            throw HeError(HE_EKEY, "no Galois key for this step");
        }
        // zero operands: the kernels' work does not depend on the values
        Tensor t;
        Ct a;
        if (step == 0) {
            t.level = level;
            t.nb = batch;
            t.buf = c.alloc((size_t)(level + 1) * 3 * c.N * batch);
            HIP_CHECK(hipMemsetAsync(t.buf->p, 0, t.buf->words * 8, c.st));
        } else {
            a = c.new_ct(level, batch);
            HIP_CHECK(hipMemsetAsync(a.d(), 0, a.buf->words * 8, c.st));
        }
        auto once = [&]() {
            if (step == 0) (void)c.relin_rescale(t, *k->k);
            else (void)c.rotate(a, step, *k->k);
        };
        once();  // warm-up: tables, caches and the pool's buffers
        std::vector<hipEvent_t> ev(reps + 1);
        for (auto &e : ev) HIP_CHECK(hipEventCreate(&e));
        std::vector<float> t_ms(reps);
        try {
            HIP_CHECK(hipEventRecord(ev[0], c.st));
            for (int r = 0; r < reps; r++) {
                once();
                HIP_CHECK(hipEventRecord(ev[r + 1], c.st));
            }
            HIP_CHECK(hipEventSynchronize(ev[reps]));
            for (int r = 0; r < reps; r++) HIP_CHECK(hipEventElapsedTime(&t_ms[r], ev[r], ev[r + 1]));
        } catch (...) {
            for (auto &e : ev) (void)hipEventDestroy(e);
            throw;
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        std::sort(t_ms.begin(), t_ms.end());
        *ms = reps % 2 ? t_ms[reps / 2] : 0.5 * (t_ms[reps / 2 - 1] + t_ms[reps / 2]);
    });
}

int he_ctx_set_keyswitch(he_ctx *ctx, int32_t level, int32_t batch, int32_t config)
{
    if (!ctx || batch < 1 || !(config == 0 || config == 1 || config == 8 || config == 32)) return HE_EINVAL;
    return guard(ctx, [&]() {
        need(level >= 0 && level <= ctx->c->L, "level out of range");
        ctx->c->ks_tune[std::make_pair((int)level, (int)batch)] = config;
    });
}

int he_ctx_profile_read(he_ctx *ctx, double *total_ms, uint64_t *launches, double *bytes, double *ops)
{
    if (!ctx) return HE_EINVAL;
    return guard(ctx, [&]() {
        double ms, b, o;
        u64 n;
        ctx->c->profile_read(ms, n, b, o);
        if (total_ms) *total_ms = ms;
        if (launches) *launches = n;
        if (bytes) *bytes = b;
        if (ops) *ops = o;
    });
}

int he_model_compile(he_ctx *ctx, const he_kan_desc *desc, int32_t refresh, he_model **out)
{
    if (!ctx || !out) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        need(desc != nullptr, "null model description");
        Model *m = new Model(ctx->c, desc, refresh != 0);
        *out = new he_model{retain(ctx), m};
    });
}

int he_model_free(he_model *m)
{
    if (!m) return HE_EINVAL;
    he_ctx *o = m->owner;
    delete m->m;
    delete m;
    release(o);
    return HE_OK;
}

int he_model_rotation_steps(const he_model *m, int32_t *steps, size_t cap, size_t *n)
{
    if (!m || !n) return HE_EINVAL;
    const auto &s = m->m->steps;
    *n = s.size();
    for (size_t i = 0; i < s.size() && i < cap && steps; i++) steps[i] = (int32_t)s[i];
    return HE_OK;
}

int he_keygen(he_ctx *ctx, uint64_t seed, const int32_t *steps, size_t nsteps, he_secret_key **sk,
              he_eval_keys **ek)
{
    if (!ctx || !sk || !ek) return HE_EINVAL;
    *sk = nullptr;
    *ek = nullptr;
    return guard(ctx, [&]() {
        need(nsteps == 0 || steps != nullptr, "null steps");
        std::vector<long> st(steps, steps + nsteps);
        SecretKey *s = nullptr;
        Keys *k = nullptr;
        ctx->c->keygen(seed, st, s, k);
        *sk = new he_secret_key{retain(ctx), s};
        *ek = new he_eval_keys{retain(ctx), k};
    });
}

int he_secret_key_free(he_secret_key *k)
{
    if (!k) return HE_EINVAL;
    he_ctx *o = k->owner;
    std::fill(k->k->s.begin(), k->k->s.end(), 0);
    delete k->k;
    delete k;
    release(o);
    return HE_OK;
}

int he_eval_keys_free(he_eval_keys *k)
{
    if (!k) return HE_EINVAL;
    he_ctx *o = k->owner;
    delete k->k;
    delete k;
    release(o);
    return HE_OK;
}

int he_eval_keys_ids(const he_eval_keys *k, uint32_t *ids, size_t cap, size_t *n)
{
    if (!k || !n || (cap && !ids)) return HE_EINVAL;
    std::vector<uint32_t> v;
    if (k->k->has_relin) v.push_back(0);
    for (auto &g : k->k->galois) v.push_back((uint32_t)g.first);
    *n = v.size();
    for (size_t i = 0; i < v.size() && i < cap; i++) ids[i] = v[i];
    return HE_OK;
}

int he_eval_keys_export(he_ctx *ctx, const he_eval_keys *k, uint32_t key_id, int32_t digit, uint64_t *out,
                        size_t cap)
{
    if (!ctx || !k || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        Ctx &c = *ctx->c;
        need(cap >= (size_t)2 * (c.L + 1 + c.alpha) * c.N, "output buffer too small");
        c.export_key(*k->k, key_id, digit, U(out));
    });
}

int he_eval_keys_import(he_ctx *ctx, const uint32_t *ids, size_t nkeys, const uint64_t *const *data,
                        he_eval_keys **out)
{
    if (!ctx || !out || (nkeys && (!ids || !data))) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        std::vector<u32> id(ids, ids + nkeys);
        std::vector<const u64 *> d;
        for (size_t i = 0; i < nkeys; i++) d.push_back(U(data[i]));
        Keys *k = ctx->c->import_keys(id, d);
        *out = new he_eval_keys{retain(ctx), k};
    });
}

int he_encrypt(he_ctx *ctx, const he_secret_key *k, const double *x, size_t n, uint64_t seed, he_ct **out)
{
    if (!ctx || !k || !out || (n && !x)) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        check_sk(ctx, k);
        *out = wrap(ctx, ctx->c->encrypt(*k->k, x, n, seed));
    });
}

int he_decrypt(he_ctx *ctx, const he_secret_key *k, const he_ct *ct, double *y, size_t n)
{
    if (!ctx || !k || !y) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_sk(ctx, k);
        check_ct(ctx, ct);
        need(n <= (size_t)ctx->c->N / 2, "too many slots requested");
        ctx->c->decrypt(*k->k, ct->c, y, n);
    });
}

int he_ct_level(const he_ct *ct) { return ct ? ct->c.level : HE_EINVAL; }

int he_ct_free(he_ct *ct)
{
    if (!ct) return HE_EINVAL;
    he_ctx *o = ct->owner;
    delete ct;
    release(o);
    return HE_OK;
}

int he_ct_export(he_ctx *ctx, const he_ct *ct, uint64_t *out, size_t cap)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, ct);
        Ctx &c = *ctx->c;
        const int nl = ct->c.level + 1;
        need(cap >= (size_t)2 * nl * c.N, "output buffer too small");
        Buf tmp = c.alloc((size_t)2 * nl * c.N);
        // [limb][2][N] NTT -> [2][limb][N] coefficient form
        launch_copy(PolySet{tmp->p, (long)c.N, (long)nl * c.N, nl, 2}, c.ctset(ct->c), c.N, c.st);
        c.ntt(PolySet{tmp->p, (long)c.N, (long)nl * c.N, nl, 2}, c.lmap(nl), true);
        c.download(U(out), tmp->p, (size_t)2 * nl * c.N);
    });
}

int he_ct_import(he_ctx *ctx, const uint64_t *in, int32_t level, he_ct **out)
{
    if (!ctx || !in || !out) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        Ctx &c = *ctx->c;
        need(level >= 0 && level <= c.L, "level out of range");
        const int nl = level + 1;
        for (int p = 0; p < 2; p++)
            for (int l = 0; l < nl; l++)
                for (int n = 0; n < c.N; n++)
                    need(in[((size_t)p * nl + l) * c.N + n] < c.q[l], "residue not reduced");
        Buf tmp = c.alloc((size_t)2 * nl * c.N);
        c.upload(tmp->p, U(in), (size_t)2 * nl * c.N);
        c.ntt(PolySet{tmp->p, (long)c.N, (long)nl * c.N, nl, 2}, c.lmap(nl), false);
        Ct o = c.new_ct(level);
        launch_copy(c.ctset(o), PolySet{tmp->p, (long)c.N, (long)nl * c.N, nl, 2}, c.N, c.st);
        *out = wrap(ctx, o);
    });
}

// n requests x nin input ciphertexts each (request-major) -> one batch per input
static std::vector<Ct> batch_inputs(he_ctx *ctx, const he_ct *const *in, size_t n, size_t nin)
{
    Ctx &c = *ctx->c;
    std::vector<Ct> xs;
    for (size_t p = 0; p < nin; p++) {
        std::vector<const Ct *> v;
        for (size_t i = 0; i < n; i++) {
            const he_ct *h = in[i * nin + p];
            check_ct(ctx, h);
            v.push_back(&h->c);
        }
        xs.push_back(n == 1 ? *v[0] : c.pack(v));
    }
    return xs;
}

static void check_model(he_ctx *ctx, const he_model *m, const he_eval_keys *k)
{
    if (m->owner != ctx) throw HeError(HE_ESTATE, "model of another context");
    check_ek(ctx, k);
}

int he_model_input_chunks(const he_model *m, int32_t *bounds, size_t cap, size_t *n)
{
    if (!m || !n) return HE_EINVAL;
    const auto &parts = m->m->layers[0].parts;
    *n = parts.size();
    for (size_t i = 0; i <= parts.size() && i < cap; i++)
        bounds[i] = i < parts.size() ? parts[i].lo : parts.back().lo + parts.back().n_in;
    return HE_OK;
}

int he_model_output_period(const he_model *m, int32_t layer, int64_t *period)
{
    if (!m || !period || layer < 0 || (size_t)layer >= m->m->layers.size()) return HE_EINVAL;
    *period = (int64_t)(m->m->layers[layer].d * m->m->S);
    return HE_OK;
}

int he_boot_create(he_ctx *ctx, const he_boot_desc *d, he_boot **out)
{
    if (!ctx || !out) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        need(d != nullptr && d->cos_coeffs != nullptr && d->cos_degree >= 1, "missing bootstrapping description");
        need(ctx->c->top < ctx->c->L, "the context has no boot levels");
        std::vector<double> cf(d->cos_coeffs, d->cos_coeffs + d->cos_degree + 1);
        need(d->real_slots == 0 || d->real_slots == 1, "real_slots must be 0 or 1");
        Boot *b = new Boot(ctx->c, d->cts_levels, d->stc_levels, d->k_range, d->double_angles, cf, d->real_slots != 0,
                           d->slots);
        *out = new he_boot{retain(ctx), b};
    });
}

int he_boot_free(he_boot *b)
{
    if (!b) return HE_EINVAL;
    he_ctx *o = b->owner;
    delete b->b;
    delete b;
    release(o);
    return HE_OK;
}

int he_boot_rotation_steps(const he_boot *b, int32_t *steps, size_t cap, size_t *n)
{
    if (!b || !n) return HE_EINVAL;
    const auto &s = b->b->steps;
    *n = s.size();
    for (size_t i = 0; i < s.size() && i < cap && steps; i++) steps[i] = (int32_t)s[i];
    return HE_OK;
}

int he_bootstrap(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *in, he_ct **out)
{
    return he_bootstrap_batch(ctx, b, k, &in, 1, out);
}

int he_bootstrap_batch(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *const *in, size_t n,
                       he_ct **out)
{
    if (!ctx || !b || !k || !out || (n && !in)) return HE_EINVAL;
    return guard(ctx, [&]() {
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
        if (n == 0) return;
        if (b->owner != ctx) throw HeError(HE_ESTATE, "bootstrapping plan of another context");
        check_ek(ctx, k);
        Ctx &c = *ctx->c;
        Ct res = bootstrap(c, *b->b, *k->k, batch_inputs(ctx, in, n, 1)[0]);
        for (size_t i = 0; i < n; i++) out[i] = wrap(ctx, n == 1 ? res : c.unpack(res, (int)i));
    });
}

int he_eval_kan_boot(he_ctx *ctx, const he_model *m, he_boot *b, const he_eval_keys *k, const he_ct *const *in,
                     size_t n, he_ct **out)
{
    if (!ctx || !m || !b || !k || !out || (n && !in)) return HE_EINVAL;
    return guard(ctx, [&]() {
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
        if (n == 0) return;
        check_model(ctx, m, k);
        if (b->owner != ctx) throw HeError(HE_ESTATE, "bootstrapping plan of another context");
        Ctx &c = *ctx->c;
        Model &md = *m->m;
        for (size_t li = 0; li + 1 < md.layers.size(); li++)
            if (b->b->slots % (md.layers[li].d * md.S) != 0)
                throw HeError(HE_ESHAPE, "the refresh keeps " + std::to_string(b->b->slots) +
                                             " slots, not a multiple of layer " + std::to_string(li) +
                                             "'s output period " + std::to_string(md.layers[li].d * md.S));
        Ct x = eval_layer(c, md, *k->k, batch_inputs(ctx, in, n, md.n_inputs()), 0);
        for (size_t li = 1; li < md.layers.size(); li++)
            x = eval_layer(c, md, *k->k, {bootstrap(c, *b->b, *k->k, x)}, li);
        for (size_t i = 0; i < n; i++) out[i] = wrap(ctx, n == 1 ? x : c.unpack(x, (int)i));
    });
}

static int boot_stage(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *in, he_ct **out, int stage,
                      int src_level)
{
    if (!ctx || !b || !k || !out) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        if (b->owner != ctx) throw HeError(HE_ESTATE, "bootstrapping plan of another context");
        check_ek(ctx, k);
        check_ct(ctx, in);
        Ctx &c = *ctx->c;
        if (stage == 0) *out = wrap(ctx, boot_coeff_to_slot(c, *b->b, *k->k, in->c));
        if (stage == 1) *out = wrap(ctx, boot_eval_mod(c, *b->b, *k->k, in->c));
        if (stage == 2) *out = wrap(ctx, boot_slot_to_coeff(c, *b->b, *k->k, in->c, src_level));
    });
}

int he_boot_coeff_to_slot(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *in, he_ct **out)
{
    return boot_stage(ctx, b, k, in, out, 0, 0);
}

int he_boot_eval_mod(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *in, he_ct **out)
{
    return boot_stage(ctx, b, k, in, out, 1, 0);
}

int he_boot_slot_to_coeff(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *in, int32_t source_level,
                          he_ct **out)
{
    return boot_stage(ctx, b, k, in, out, 2, source_level);
}

int he_eval_kan(he_ctx *ctx, const he_model *m, const he_eval_keys *k, const he_ct *in, he_ct **out)
{
    return he_eval_kan_chunks(ctx, m, k, &in, 1, out);
}

int he_eval_kan_chunks(he_ctx *ctx, const he_model *m, const he_eval_keys *k, const he_ct *const *in, size_t n_in,
                       he_ct **out)
{
    if (!ctx || !m || !k || !out || !in) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        check_model(ctx, m, k);
        if (n_in != m->m->n_inputs())
            throw HeError(HE_ESHAPE, "the model takes " + std::to_string(m->m->n_inputs()) + " input ciphertexts");
        *out = wrap(ctx, eval_model(*ctx->c, *m->m, *k->k, batch_inputs(ctx, in, 1, n_in)));
    });
}

int he_eval_kan_layer(he_ctx *ctx, const he_model *m, const he_eval_keys *k, int32_t layer, const he_ct *in,
                      he_ct **out)
{
    if (!ctx || !m || !k || !out) return HE_EINVAL;
    *out = nullptr;
    return he_eval_kan_layer_batch(ctx, m, k, layer, &in, 1, out);
}

int he_eval_kan_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *k, const he_ct *const *in, size_t n,
                      he_ct **out)
{
    if (!ctx || !m || !k || !out || (n && !in)) return HE_EINVAL;
    return guard(ctx, [&]() {
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
        if (n == 0) return;
        check_model(ctx, m, k);
        Ctx &c = *ctx->c;
        Ct res = eval_model(c, *m->m, *k->k, batch_inputs(ctx, in, n, m->m->n_inputs()));
        for (size_t i = 0; i < n; i++) out[i] = wrap(ctx, n == 1 ? res : c.unpack(res, (int)i));
    });
}

int he_eval_kan_layer_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *k, int32_t layer,
                            const he_ct *const *in, size_t n, he_ct **out)
{
    if (!ctx || !m || !k || !out || (n && !in)) return HE_EINVAL;
    return guard(ctx, [&]() {
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
        if (n == 0) return;
        check_model(ctx, m, k);
        need(layer >= 0 && (size_t)layer < m->m->layers.size(), "layer out of range");
        const size_t nin = layer == 0 ? m->m->n_inputs() : 1;
        Ctx &c = *ctx->c;
        Ct res = eval_layer(c, *m->m, *k->k, batch_inputs(ctx, in, n, nin), (size_t)layer);
        for (size_t i = 0; i < n; i++) out[i] = wrap(ctx, n == 1 ? res : c.unpack(res, (int)i));
    });
}

// Capture `run` (which issues the work on the context stream and returns its
// n outputs) into a graph: one eager run fills every cache and leaves the pool
// holding the buffers a run needs, so the captured run makes no host transfer
// and no synchronisation; the graph keeps `inputs` and the outputs alive and
// owns its temporaries until it is freed.
static void capture_graph(he_ctx *ctx, const std::function<std::vector<Ct>()> &run, const std::vector<Ct> &inputs,
                          size_t n, he_ct **out, he_graph **g)
{
    Ctx &c = *ctx->c;
    { std::vector<Ct> warm = run(); }
    c.sync();
    std::unique_ptr<he_graph> gr(new he_graph);
    gr->owner = ctx;  // retained once the graph is complete
    const int timer = c.timer.target;
    c.timer.target = -1;
    c.pool.hold = &gr->held;
    std::vector<Ct> outs;
    HIP_CHECK(hipStreamBeginCapture(c.st, hipStreamCaptureModeRelaxed));
    try {
        outs = run();
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(c.st, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        c.pool.hold = nullptr;
        c.timer.target = timer;
        for (auto &h : gr->held) c.pool.free_.emplace(h.first, h.second), c.pool.cached += h.first;
        throw;
    }
    c.pool.hold = nullptr;
    c.timer.target = timer;
    // the graph's temporaries count as live memory until the graph is freed
    for (auto &h : gr->held) c.pool.live += h.first;
    const hipError_t ec = hipStreamEndCapture(c.st, &gr->graph);
    if (ec != hipSuccess || !gr->graph) {
        for (auto &h : gr->held) c.pool.put(h.second, h.first);
        throw HeError(HE_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ec));
    }
    HIP_CHECK(hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0));
    // captured launches were recorded, not run: one launch computes the outputs
    HIP_CHECK(hipGraphLaunch(gr->exec, c.st));
    for (const Ct &x : inputs) gr->keep.push_back(x);
    for (auto &o : outs) gr->keep.push_back(o);
    for (size_t i = 0; i < n; i++) out[i] = wrap(ctx, outs[i]);
    retain(ctx);
    *g = gr.release();
}

int he_graph_capture_kan_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *k, const he_ct *const *in, size_t n,
                               he_ct **out, he_graph **g)
{
    if (!ctx || !m || !k || !out || !g || !in || n == 0) return HE_EINVAL;
    *g = nullptr;
    for (size_t i = 0; i < n; i++) out[i] = nullptr;
    return guard(ctx, [&]() {
        check_model(ctx, m, k);
        Ctx &c = *ctx->c;
        const size_t nin = m->m->n_inputs();
        std::vector<Ct> inputs;
        for (size_t i = 0; i < n * nin; i++) {
            check_ct(ctx, in[i]);
            inputs.push_back(in[i]->c);
        }
        auto run = [&]() {
            Ct res = eval_model(c, *m->m, *k->k, batch_inputs(ctx, in, n, nin));
            std::vector<Ct> o;
            for (size_t i = 0; i < n; i++) o.push_back(n == 1 ? res : c.unpack(res, (int)i));
            return o;
        };
        capture_graph(ctx, run, inputs, n, out, g);
    });
}

int he_graph_capture_bootstrap(he_ctx *ctx, he_boot *b, const he_eval_keys *k, const he_ct *const *in, size_t n,
                               he_ct **out, he_graph **g)
{
    if (!ctx || !b || !k || !out || !g || !in || n == 0) return HE_EINVAL;
    *g = nullptr;
    for (size_t i = 0; i < n; i++) out[i] = nullptr;
    return guard(ctx, [&]() {
        if (b->owner != ctx) throw HeError(HE_ESTATE, "bootstrapping plan of another context");
        check_ek(ctx, k);
        Ctx &c = *ctx->c;
        std::vector<Ct> inputs;
        for (size_t i = 0; i < n; i++) {
            check_ct(ctx, in[i]);
            inputs.push_back(in[i]->c);
        }
        auto run = [&]() {
            Ct res = bootstrap(c, *b->b, *k->k, batch_inputs(ctx, in, n, 1)[0]);
            std::vector<Ct> o;
            for (size_t i = 0; i < n; i++) o.push_back(n == 1 ? res : c.unpack(res, (int)i));
            return o;
        };
        capture_graph(ctx, run, inputs, n, out, g);
    });
}

int he_graph_launch(he_graph *g)
{
    if (!g) return HE_EINVAL;
    return guard(g->owner, [&]() { HIP_CHECK(hipGraphLaunch(g->exec, g->owner->c->st)); });
}

int he_graph_free(he_graph *g)
{
    if (!g) return HE_EINVAL;
    he_ctx *o = g->owner;
    const int rc = guard(o, [&]() { o->c->sync(); });
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (auto &h : g->held) o->c->pool.put(h.second, h.first);
    g->keep.clear();
    delete g;
    release(o);
    return rc;
}

int he_ctx_memory(he_ctx *ctx, uint64_t *live, uint64_t *cached, uint64_t *peak, int32_t reset_peak)
{
    if (!ctx) return HE_EINVAL;
    Pool &p = ctx->c->pool;
    if (live) *live = p.live;
    if (cached) *cached = p.cached;
    if (peak) *peak = p.peak;
    if (reset_peak) p.peak = p.live;
    return HE_OK;
}

int he_ctx_device_memory(he_ctx *ctx, uint64_t *free_bytes, uint64_t *total_bytes)
{
    if (!ctx) return HE_EINVAL;
    return guard(ctx, [&]() {
        size_t f = 0, t = 0;
        HIP_CHECK(hipMemGetInfo(&f, &t));
        if (free_bytes) *free_bytes = f;
        if (total_bytes) *total_bytes = t;
    });
}

int he_ct_add(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        check_ct(ctx, b);
        *out = wrap(ctx, ctx->c->add(a->c, b->c));
    });
}

int he_ct_mul(he_ctx *ctx, const he_eval_keys *k, const he_ct *a, const he_ct *b, he_ct **out)
{
    if (!ctx || !k || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        check_ct(ctx, a);
        check_ct(ctx, b);
        need(a->c.level == b->c.level, "operands at different levels");
        need(a->c.level >= 1, "no level left");
        *out = wrap(ctx, ctx->c->mul(a->c, b->c, *k->k));
    });
}

int he_ct_rotate(he_ctx *ctx, const he_eval_keys *k, const he_ct *a, int32_t step, he_ct **out)
{
    if (!ctx || !k || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        check_ct(ctx, a);
        *out = wrap(ctx, ctx->c->rotate(a->c, step, *k->k));
    });
}

int he_ct_rotate_sum(he_ctx *ctx, const he_eval_keys *k, const he_ct *const *in, const int32_t *steps, size_t n,
                     he_ct **out)
{
    if (!ctx || !k || !out || !in || !steps || n == 0) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        check_ek(ctx, k);
        std::vector<std::pair<const Ct *, long>> items;
        for (size_t i = 0; i < n; i++) {
            check_ct(ctx, in[i]);
            if (in[i]->c.level != in[0]->c.level || in[i]->c.nb != in[0]->c.nb)
                throw HeError(HE_ESHAPE, "rotate_sum: the ciphertexts differ in level or batch size");
            items.push_back({&in[i]->c, (long)steps[i]});
        }
        *out = wrap(ctx, ctx->c->rotate_sum(items, *k->k));
    });
}

int he_ct_sub(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        check_ct(ctx, b);
        *out = wrap(ctx, ctx->c->sub(a->c, b->c));
    });
}

int he_ct_mod_drop(he_ctx *ctx, const he_ct *a, int32_t level, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        need(level >= 0 && level <= a->c.level, "mod_drop: level out of range");
        *out = wrap(ctx, ctx->c->mod_drop(a->c, level));
    });
}

int he_ct_mul_i(he_ctx *ctx, const he_ct *a, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        *out = wrap(ctx, ctx->c->mul_i(a->c));
    });
}

int he_ct_mod_raise(he_ctx *ctx, const he_ct *a, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        need(a->c.level == 0, "mod_raise: the input must be at level 0");
        *out = wrap(ctx, ctx->c->mod_raise(a->c));
    });
}

int he_ct_rescale(he_ctx *ctx, const he_ct *a, he_ct **out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        *out = wrap(ctx, ctx->c->rescale(a->c));
    });
}

int he_ct_rescale_noalloc(he_ctx *ctx, const he_ct *a, he_ct *out)
{
    if (!ctx || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        check_ct(ctx, a);
        check_ct(ctx, out);
        Ctx &c = *ctx->c;
        need(a->c.nb == 1 && out->c.nb == 1, "batched ciphertext");
        if (a->c.level < 1) throw HeError(HE_EDEPTH, "rescale: no level left");
        need(out->c.level == a->c.level - 1, "output level must be the input level - 1");
        const size_t need_words = (size_t)(a->c.level + 1) * 2 * c.N;
        if (need_words * sizeof(u64) > kNoAllocScratchBytes)
            throw HeError(HE_ENOMEM, "rescale of " + std::to_string(a->c.level + 1) + " limbs of N = " +
                                         std::to_string(c.N) + " needs " + std::to_string(need_words * 8) +
                                         " bytes of scratch, more than the " +
                                         std::to_string(kNoAllocScratchBytes) + " the library holds");
        const u64 *ab = a->c.buf->p, *ob = out->c.buf->p;
        const size_t aw = (size_t)(a->c.level + 1) * 2 * c.N, ow = (size_t)(out->c.level + 1) * 2 * c.N;
        need(ob + ow <= ab || ab + aw <= ob, "output shares memory with the input");
        // another handle (a rotation by 0 returns its input's memory) or a
        // graph holding the same buffer would see its residues overwritten
        need(out->c.buf.use_count() == 1, "output shares memory with another ciphertext");
        if (!c.scratch) throw HeError(HE_ESTATE, "no scratch on this device");
        c.rescale_into(a->c, out->c, c.scratch);
    });
}

int he_ct_lincomb(he_ctx *ctx, const he_ct *const *a, size_t n, const double *z, size_t n_slots, int32_t target,
                  he_ct **out)
{
    if (!ctx || !out || !a || !z || n == 0) return HE_EINVAL;
    return guard(ctx, [&]() {
        Ctx &c = *ctx->c;
        need(target >= 0, "bad target level");
        std::vector<Pt> pts(n);
        std::vector<std::pair<const Ct *, const Pt *>> terms;
        for (size_t i = 0; i < n; i++) {
            check_ct(ctx, a[i]);
            need(a[i]->c.level >= target + 1, "operand below target + 1");
            double X = c.S[target] * (double)c.q[target + 1] / c.S[a[i]->c.level];
            if (n_slots == 1) pts[i] = c.const_pt(z[i], X, target + 2);
            else pts[i] = c.vec_pt(z + i * n_slots, n_slots, X, target + 2);
        }
        for (size_t i = 0; i < n; i++) terms.push_back({&a[i]->c, &pts[i]});
        *out = wrap(ctx, c.lincomb(terms, target));
    });
}

int he_poly_mul(he_ctx *ctx, const uint64_t *a, const uint64_t *b, int32_t nl, uint64_t *out)
{
    if (!ctx || !a || !b || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        Ctx &c = *ctx->c;
        need(nl >= 1 && nl <= c.L + 1, "limb count out of range");
        size_t words = (size_t)nl * c.N;
        Buf da = c.alloc(words), db = c.alloc(words);
        c.upload(da->p, U(a), words);
        c.upload(db->p, U(b), words);
        PolySet pa{da->p, (long)c.N, 0, nl, 1}, pb{db->p, (long)c.N, 0, nl, 1};
        LimbMap lm = c.lmap(nl);
        c.ntt(pa, lm, false);
        c.ntt(pb, lm, false);
        launch_pmul(c.d_pc, pa, pa, pb, lm, c.N, c.st);
        c.ntt(pa, lm, true);
        c.download(U(out), da->p, words);
    });
}

int he_encode(he_ctx *ctx, const double *z, size_t n, double scale, int32_t nl, uint64_t *out)
{
    if (!ctx || (n && !z) || !out) return HE_EINVAL;
    return guard(ctx, [&]() {
        Ctx &c = *ctx->c;
        need(nl >= 1 && nl <= (int)c.mods.size(), "limb count out of range");
        need(n <= (size_t)c.N / 2, "too many slots");
        encode_rns(z, n, scale, c.logN, c.mods.data(), nl, U(out));
    });
}

}  // extern "C"
