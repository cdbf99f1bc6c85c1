// Native continuous-batching server over one context (he_server_create,
// he_submit, he_poll, he_server_stats, he_server_destroy in include/hekan.h).
//
// A worker thread owned by the server runs every submitted request layer by
// layer.  It admits requests in submission order while their models' working
// memory fits the budget, then repeatedly evaluates the (model, layer) group
// of the oldest admitted request as one batch (every ring kernel covering
// the whole group), so requests submitted while others run share launches
// with them.  A model's working memory (the pool's peak growth over one
// request) is measured on its first request, which runs alone.  Results
// wait in the server until he_poll takes them.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <set>
#include <thread>

#include "handles.hpp"

namespace {
typedef std::chrono::steady_clock Clock;

struct Req {
    uint64_t tag = 0;
    const he_model *m = nullptr;
    std::vector<Ct> x;  // the input chunks, then the latest layer's output
    size_t layer = 0;
    uint64_t need = 0;  // bytes charged against the budget while admitted
    bool measure = false;
    uint64_t live0 = 0;
    Clock::time_point t_submit;
};

struct Result {
    int code = HE_OK;
    Ct ct;
    double latency_ms = 0.0;
};
}  // namespace

struct he_server {
    he_ctx *ctx;
    const he_eval_keys *ek;
    int max_batch;
    uint64_t budget;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> queue;
    std::vector<Req> active;                   // in admission order
    std::map<uint64_t, Result> results;
    std::set<uint64_t> pending;                 // submitted, not finished
    std::map<const he_model *, uint64_t> work;  // measured working bytes per model
    uint64_t next_tag = 1, in_use = 0;
    uint64_t n_done = 0, n_batches = 0, n_runs = 0;
    bool stop = false;
    std::thread worker;
    void run();
    void step(std::unique_lock<std::mutex> &lk);
};

void he_server::run()
{
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // admission in submission order: a request enters while its model's
        // working memory fits the budget; a model's first request runs alone
        while (!queue.empty()) {
            Req &r = queue.front();
            auto w = work.find(r.m);
            const bool known = w != work.end();
            if (!active.empty() && (!known || in_use + w->second > budget)) break;
            r.need = known ? w->second : 0;
            r.measure = !known;
            in_use += r.need;
            active.push_back(std::move(r));
            queue.pop_front();
            if (!known) break;
        }
        if (active.empty()) {
            if (stop) return;
            cv.wait(lk);
            continue;
        }
        step(lk);
    }
}

// One layer for the oldest admitted request's (model, layer) group, batched.
// The GPU work runs outside the lock; only this thread touches `active`.
void he_server::step(std::unique_lock<std::mutex> &lk)
{
    const he_model *m = active[0].m;
    const size_t layer = active[0].layer;
    std::vector<size_t> idx;
    for (size_t i = 0; i < active.size() && (int)idx.size() < max_batch; i++)
        if (active[i].m == m && active[i].layer == layer) idx.push_back(i);
    const bool measure = active[idx[0]].measure;
    lk.unlock();
    Ctx &c = *ctx->c;
    int code = HE_OK;
    std::vector<Ct> outs;
    try {
        (void)hipGetLastError();
        if (measure && layer == 0) {
            c.sync();
            active[idx[0]].live0 = c.pool.live;
            c.pool.peak = c.pool.live;
        }
        const size_t nin = active[idx[0]].x.size(), n = idx.size();
        std::vector<Ct> xs;
        for (size_t p = 0; p < nin; p++) {
            std::vector<const Ct *> v;
            for (size_t i : idx) v.push_back(&active[i].x[p]);
            xs.push_back(n == 1 ? *v[0] : c.pack(v));
        }
        Ct res = eval_layer(c, *m->m, *ek->k, xs, layer);
        for (size_t i = 0; i < n; i++) outs.push_back(n == 1 ? res : c.unpack(res, (int)i));
        c.sync();
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess) throw HipError(std::string("kernel launch failed: ") + hipGetErrorString(le));
    } catch (const HeError &e) {
        code = e.code;
    } catch (const HipError &) {
        code = HE_EDEVICE;
    } catch (const std::bad_alloc &) {
        code = HE_ENOMEM;
    } catch (...) {
        code = HE_EINVAL;
    }
    lk.lock();
    n_batches++;
    n_runs += idx.size();
    const Clock::time_point now = Clock::now();
    const size_t nl = m->m->layers.size();
    std::vector<size_t> finished;
    for (size_t j = 0; j < idx.size(); j++) {
        Req &r = active[idx[j]];
        if (code == HE_OK) {
            r.x.assign(1, outs[j]);
            r.layer++;
        }
        if (code != HE_OK || r.layer == nl) {
            Result res;
            res.code = code;
            if (code == HE_OK) res.ct = r.x[0];
            res.latency_ms = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
            if (r.measure && code == HE_OK) work[r.m] = std::max<uint64_t>(c.pool.peak - r.live0, 1);
            results[r.tag] = std::move(res);
            pending.erase(r.tag);
            in_use -= r.need;
            n_done++;
            finished.push_back(idx[j]);
        }
    }
    for (size_t k = finished.size(); k-- > 0;) active.erase(active.begin() + (long)finished[k]);
    cv.notify_all();
}

extern "C" {

int he_server_create(he_ctx *ctx, const he_eval_keys *ek, int32_t max_batch, uint64_t hbm_budget, he_server **out)
{
    if (!ctx || !ek || !out || max_batch < 1) return HE_EINVAL;
    *out = nullptr;
    return guard(ctx, [&]() {
        check_ek(ctx, ek);
        he_server *s = new he_server();
        s->ctx = retain(ctx);
        s->ek = ek;
        s->max_batch = max_batch;
        s->budget = hbm_budget;
        s->worker = std::thread([s]() { s->run(); });
        *out = s;
    });
}

int he_submit(he_server *s, const he_model *m, const he_ct *const *in, size_t n_in, uint64_t *tag)
{
    if (!s || !m || !tag || (n_in && !in)) return HE_EINVAL;
    return guard(s->ctx, [&]() {
        if (m->owner != s->ctx) throw HeError(HE_ESTATE, "model of another context");
        if (n_in != m->m->n_inputs())
            throw HeError(HE_ESHAPE, "the model takes " + std::to_string(m->m->n_inputs()) + " input ciphertexts");
        Req r;
        r.m = m;
        for (size_t i = 0; i < n_in; i++) {
            check_ct(s->ctx, in[i]);
            need(in[i]->c.nb == 1, "batched ciphertext");
            need(in[i]->c.level == in[0]->c.level, "input chunks at different levels");
            r.x.push_back(in[i]->c);
        }
        r.t_submit = Clock::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop) throw HeError(HE_ESTATE, "server is shutting down");
            r.tag = s->next_tag++;
            *tag = r.tag;
            s->pending.insert(r.tag);
            s->queue.push_back(std::move(r));
        }
        s->cv.notify_all();
    });
}

int he_poll(he_server *s, uint64_t tag, int32_t wait_ms, he_ct **out, double *latency_ms)
{
    if (!s || !out) return HE_EINVAL;
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    const Clock::time_point until = Clock::now() + std::chrono::milliseconds(wait_ms > 0 ? wait_ms : 0);
    for (;;) {
        auto it = s->results.find(tag);
        if (it != s->results.end()) {
            const int code = it->second.code;
            if (latency_ms) *latency_ms = it->second.latency_ms;
            if (code == HE_OK) *out = wrap(s->ctx, it->second.ct);
            s->results.erase(it);
            return code;
        }
        if (!s->pending.count(tag)) return HE_EINVAL;  // never submitted, or already taken
        if (wait_ms <= 0 || s->cv.wait_until(lk, until) == std::cv_status::timeout) {
            if (s->results.count(tag)) continue;
            return HE_EAGAIN;
        }
    }
}

int he_server_stats(he_server *s, uint64_t *completed, uint64_t *layer_batches, uint64_t *layer_runs)
{
    if (!s) return HE_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (completed) *completed = s->n_done;
    if (layer_batches) *layer_batches = s->n_batches;
    if (layer_runs) *layer_runs = s->n_runs;
    return HE_OK;
}

int he_server_destroy(he_server *s)
{
    if (!s) return HE_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
    he_ctx *o = s->ctx;
    delete s;
    release(o);
    return HE_OK;
}

}  // extern "C"
