// Internal to the library: the structs behind the opaque handles of
// include/hekan.h and the helpers every extern "C" entry point uses (error
// capture, handle ownership checks, context reference counting).
#pragma once
#include <atomic>
#include <map>
#include <string>
#include <vector>

#include "../../include/hekan.h"
#include "boot.hpp"
#include "ckks.hpp"
#include "kan.hpp"

using namespace hk;

// A context lives until it has been destroyed and every handle made from it
// has been freed (each handle holds one reference, the caller one more).
struct he_ctx {
    Ctx *c;
    std::string err;
    std::atomic<long> refs{1};
};
struct he_model {
    he_ctx *owner;
    Model *m;
};
struct he_boot {
    he_ctx *owner;
    Boot *b;
};
struct he_secret_key {
    he_ctx *owner;
    SecretKey *k;
};
struct he_eval_keys {
    he_ctx *owner;
    Keys *k;
};
struct he_ct {
    he_ctx *owner;
    Ct c;
};
struct he_graph {
    he_ctx *owner;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Ct> keep;                          // inputs and outputs the graph reads and writes
    std::multimap<size_t, void *> held;           // temporaries, owned until the graph is freed
};

namespace {
he_ctx *retain(he_ctx *h)
{
    h->refs.fetch_add(1);
    return h;
}

void release(he_ctx *h)
{
    if (h->refs.fetch_sub(1) == 1) {
        delete h->c;
        delete h;
    }
}

template <class F>
int guard(he_ctx *ctx, F f)
{
    try {
        // a launch that fails (a grid the device rejects) leaves its error to be
        // read back: clear what an earlier caller left and check after the call
        (void)hipGetLastError();
        f();
        const hipError_t le = hipGetLastError();
        if (le != hipSuccess) throw HipError(std::string("kernel launch failed: ") + hipGetErrorString(le));
        return HE_OK;
    } catch (const HeError &e) {
        if (ctx) ctx->err = e.what();
        return e.code;
    } catch (const HipError &e) {
        if (ctx) ctx->err = e.what();
        return HE_EDEVICE;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = "host allocation failed";
        return HE_ENOMEM;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = e.what();
        return HE_EINVAL;
    } catch (...) {
        if (ctx) ctx->err = "unknown error";
        return HE_EINVAL;
    }
}

void need(bool ok, const char *msg)
{
    if (!ok) throw HeError(HE_EINVAL, msg);
}

he_ct *wrap(he_ctx *ctx, Ct c)
{
    he_ct *h = new he_ct();
    h->owner = retain(ctx);
    h->c = std::move(c);
    return h;
}

inline u64 *U(uint64_t *p) { return reinterpret_cast<u64 *>(p); }
inline const u64 *U(const uint64_t *p) { return reinterpret_cast<const u64 *>(p); }

void check_ct(he_ctx *ctx, const he_ct *c)
{
    need(c != nullptr, "null ciphertext");
    if (c->owner != ctx) throw HeError(HE_ESTATE, "ciphertext belongs to another context");
}

void check_ek(he_ctx *ctx, const he_eval_keys *k)
{
    need(k != nullptr, "null evaluation keys");
    if (k->owner != ctx) throw HeError(HE_ESTATE, "evaluation keys of another context");
}

void check_sk(he_ctx *ctx, const he_secret_key *k)
{
    need(k != nullptr, "null secret key");
    if (k->owner != ctx) throw HeError(HE_ESTATE, "secret key of another context");
}
}  // namespace
