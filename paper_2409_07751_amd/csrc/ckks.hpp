// Device-resident RNS-CKKS: context, ciphertexts, keys and homomorphic ops.
#pragma once
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "dev.hpp"
#include "hostmath.hpp"

namespace hk {

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct HeError : std::runtime_error {
    int code;
    HeError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(x)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess)                                                                 \
            throw ::hk::HipError(std::string(#x) + ": " + hipGetErrorString(e_));             \
    } while (0)

struct Ctx;

// The rotation "step" that names the complex conjugation (Galois element 2N - 1).
constexpr long kStepConjugate = -(1l << 31);

// Size of the device array behind the entry points that allocate nothing (one
// copy per device), and its set-up: looks up the array's device address for
// the current device (once per device) and returns it.
constexpr size_t kNoAllocScratchBytes = 32ull << 20;
u64 *noalloc_scratch_setup();

// Caching device allocator: buffers go back to per-size free lists and are
// reused in stream order (all work of a context runs on one stream).
struct Pool {
    std::multimap<size_t, void *> free_;
    size_t live = 0, cached = 0, peak = 0;
    // while a graph is being captured, buffers released go to this list
    // instead of the shared one: the capture reuses them (its launches run in
    // order), and afterwards the graph owns them until it is destroyed
    std::multimap<size_t, void *> *hold = nullptr;
    void *get(size_t bytes);
    void put(void *p, size_t bytes);
    void trim();
    ~Pool();
};

struct DevBuf {
    Ctx *ctx;
    u64 *p;
    size_t words;
    ~DevBuf();
};
typedef std::shared_ptr<DevBuf> Buf;

// Ciphertext: level l, [l+1][2][N] residues in NTT form (limb-major, c0 then
// c1 inside each limb), scale = canonical S[l].
// A batch of nb ciphertexts is [l+1][nb][2][N]: every launch covers all of them.
struct Ct {
    int level = -1;
    int nb = 1;
    Buf buf;
    u64 *d() const { return buf->p; }
};

// Tensor product (d0, d1, d2) before relinearisation: [l+1][3][N].
struct Tensor {
    int level = -1;
    int nb = 1;
    Buf buf;
};

// Plaintext for a linear combination: a constant (per-limb residues) or a
// slot vector (NTT form), both in Montgomery form, covering >= nl limbs.
struct Pt {
    Buf buf;
    bool is_const = false;
    int nl = 0;
    // constants only: [4][L+1] the residues C_i, their Shoup words, C_i N^-1
    // and its Shoup words (standard form, for products folded into a rescale)
    Buf plain;
};

struct SwitchKey {
    Buf buf;   // [dnum][2][L+1+alpha][N] NTT + Montgomery form
    Buf fbuf;  // the same layout in standard form as doubles, filled on FP64 primes (fused ModUp products)
};

// Evaluation keys (server side): no secret material.
struct Keys {
    Ctx *ctx;
    SwitchKey relin;
    bool has_relin = false;
    std::map<u64, SwitchKey> galois;
};

// The ternary secret, in host memory (client side).
struct SecretKey {
    Ctx *ctx;
    std::vector<int64_t> s;
};

// per-level key-switch constants: [2][nq] INTT output scale (inverse hat of
// the limb's digit times N^-1, Shoup pair) then [ndig][w][nq+alpha] ModUp
// conversion constants (Montgomery form)
struct KsTable {
    Buf buf, fbuf;
    const u64 *scale, *scalep, *hatm;
    const TwF *hatf;  // hatm in standard form as FP64 pairs (entries for FP64 targets)
    const TwF *scalef;  // [nq] scale as FP64 pairs (entries for FP64 primes)
    u64 wide[2];      // bit 8 j + k: source k of digit j is a prime above 2^50
    u64 dbl[2];       // bit 8 j + k: source k of digit j is an FP64 prime (held as a double)
};

struct Ctx {
    int logN, N, L, alpha, w, L1;
    int top;      // top computation level: L minus the levels kept for bootstrapping
    int hamming;  // Hamming weight of a sparse ternary secret (0: uniform ternary)
    double sigma;
    std::vector<u64> q, p, mods;  // mods = q ++ p
    std::vector<double> S;
    std::vector<PrimeConst> pc;
    hipStream_t st = nullptr;
    bool own_stream = false;
    Pool pool;
    Buf d_pc_buf, tw_buf, twf_buf, twab_buf;
    const PrimeConst *d_pc = nullptr;
    NttTables T;
    std::map<int, KsTable> ks_cache;
    std::map<std::pair<int, long>, Buf> rescale_inv;  // per (level l, factor k): [2][l] k q_l^-1, Shoup
    std::map<std::tuple<int, long, u64>, Buf> rescale_add;  // per (l, k, constant bits): [l] pre-rescale addend
    Buf pinv;                        // [2][L+1] P^-1 mod q_i and Shoup
    Buf pmod;                        // [2][L+1] P mod q_i and Shoup, then [L+1] FP64 pairs
    Buf md_tab;                      // [2][alpha] P-limb INTT scale, then [alpha][L+1] P->Q constants
    std::map<std::pair<u64, u64>, Buf> const_cache;
    std::map<std::pair<u64, u64>, Buf> const_plain_cache;
    std::map<int, Buf> int_cache;
    std::string err;
    u64 n_ks = 0, n_rescale = 0, n_launch = 0;
    // q_fp_lo..q_fp_top: the run of FP64 primes at the bottom of the chain
    // (fp_lo = 0 if q_0 is below 2^46, else 1; fp_top = L unless the chain
    // keeps wider boot levels on top): single key switches fuse the key inner
    // product into ModUp's second pass on those limbs; the other limbs (q_0
    // when it is wide, wider primes above q_fp_top, the special primes) take
    // the stored second pass and the separate inner product
    bool ks_fused = false;
    int fp_lo = 1, fp_top = 0;
    KernelTimer timer;
    void profile(int kernel_id);  // -1 disables; clears previous records
    void profile_read(double &ms, u64 &launches, double &bytes, double &ops);

    Ctx(int logN, int L, int scale_bits, int base_bits, int alpha, int special_bits, int w, double sigma,
        hipStream_t stream, bool integer_words = false, int boot_levels = 0, int boot_bits = 0, int hamming = 0);
    ~Ctx();

    Buf alloc(size_t words);
    int dnum_top() const { return (L + 1 + w - 1) / w; }
    int ndig(int l) const { return (l + 1 + w - 1) / w; }
    LimbMap lmap(int nq) const { return LimbMap{nq, L1}; }
    u64 galois_elt(long step) const;

    // polynomial helpers
    void ntt(PolySet ps, LimbMap lm, bool inverse, int skip_lo = 0, int skip_hi = 0);
    PolySet ctset(const Ct &c, int nl = -1) const;  // all 2 nb polynomials
    PolySet c0set(const Ct &c) const;              // the nb c0 polynomials (c1 at +N)

    // ciphertext ops (every result has canonical scale S[level])
    Ct new_ct(int level, int nb = 1);
    Ct add(const Ct &a, const Ct &b);
    Ct sub(const Ct &a, const Ct &b);
    Ct mul_int(const Ct &a, long k);
    Ct add_const(const Ct &a, double c);
    Ct add_plain(const Ct &a, const Buf &pt_ntt);  // pt in NTT standard form over >= level+1 limbs
    // k a [+ *c | + *pt] in one pass; same residues as mul_int then add_const / add_plain
    Ct affine(const Ct &a, long k, const double *c, const Buf *pt);
    Ct mod_drop(const Ct &a, int l) const;
    // ModRaise of a level-0 ciphertext: its residues mod q_0 as centred
    // integers, lifted to every prime of level L
    Ct mod_raise(const Ct &a);
    // every slot times i: the product with the monomial X^(N/2) (exact)
    Ct mul_i(const Ct &a);
    Buf mono_half;  // NTT of X^(N/2) over the L+1 Q primes
    Ct rescale(const Ct &a);
    // k rescale(a) [+ c]: the integer factor and the constant (at the result's
    // scale) are applied in the rescale's last pass; same residues as
    // add_const(mul_int(rescale(a), k), c)
    Ct rescale_affine(const Ct &a, long k, const double *c);
    // rescale(a) into the existing single ciphertext o (level a.level - 1),
    // staging through `scr` ((a.level + 1) 2 N words): no allocation; the
    // level's table must exist (the constructor builds every level's)
    void rescale_into(const Ct &a, Ct &o, u64 *scr);
    u64 *scratch = nullptr;  // this device's no-allocation scratch (kNoAllocScratchBytes)
    // rescale to level t of C a (C the constant plaintext pt, a at level >= t + 1) [+ c]:
    // the product happens in the rescale's passes; same residues as
    // rescale(lincomb({a, pt}, t)) [+ c]
    Ct rescale_const_mul(const Ct &a, const Pt &pt, int t, const double *c);
    Tensor tensor(const Ct &a, const Ct &b);
    void tensor_acc(Tensor &t, const Ct &a, const Ct &b);
    Ct relin_rescale(const Tensor &t, const Keys &k, long mul = 1, const double *c = nullptr);
    Ct mul(const Ct &a, const Ct &b, const Keys &k);
    // k (a b) [+ c] with the factor and constant folded into the rescale
    Ct mul_affine(const Ct &a, const Ct &b, const Keys &keys, long k, const double *c);
    Ct rotate(const Ct &a, long step, const Keys &k);
    // addend + rot(a, step) in one key switch (the addition runs in ModDown's last pass)
    Ct rotate_add(const Ct &a, long step, const Ct &addend, const Keys &k);
    // sum_i rot(x_i, step_i) (one level and batch) with a single ModDown: the
    // rotations' key-switch accumulators, permuted, are added over Q_l u P and
    // divided by P once; the rotated c_0 parts and the unrotated terms add in
    // Q_l (differs from the separate rotations only by ModDown's rounding)
    Ct rotate_sum(const std::vector<std::pair<const Ct *, long>> &items, const Keys &k);
    // sum of ciphertext x plaintext terms, rescaled to level t [+ the constant *c, added in the rescale]
    Ct lincomb(const std::vector<std::pair<const Ct *, const Pt *>> &terms, int t, const double *c = nullptr);
    Ct level_down(const Ct &a, int t);

    // key switching of d (NTT form, limb stride ls, level l) into out = base + KS(d);
    // the ModUp part can be shared by several keys (hoisted rotations)
    struct ModUp {
        const u64 *d = nullptr;
        long ls = 0, es = 0;
        int l = -1, nb = 1;
        Buf ext;
    };
    ModUp modup(const u64 *d, long ls, long es, int l, int nb);
    // out = base (masked components, component 0 through sigma) + KS(d) [+ addend]
    void keyswitch_from(const ModUp &m, const SwitchKey &key, u64 galois, const u64 *base, long base_ls,
                        long base_es, int base_mask, Ct &out, const Ct *addend = nullptr);
    void keyswitch(const u64 *d, long ls, long es, int l, int nb, const SwitchKey &key, u64 galois,
                   const u64 *base, long base_ls, long base_es, int base_mask, Ct &out,
                   const Ct *addend = nullptr);
    // ModDown of the accumulators acc [nb][2][l+1+alpha][N] into out (base and addend as in keyswitch_from)
    void moddown_into(const Buf &acc, int l, int nb, u64 galois, const u64 *base, long base_ls, long base_es,
                      int base_mask, Ct &out, const Ct *addend);
    // ModUp and inner product of a key switch (the accumulators before ModDown)
    Buf keyswitch_acc(const u64 *d, long ls, long es, int l, int nb, const SwitchKey &key);
    // key-switch configuration per (level, batch size): 0 ModUp then inner
    // product; 1, 8, 32 the fused kernel with that block span (default 8)
    std::map<std::pair<int, int>, int> ks_tune;
    std::vector<int> autotune_keyswitch(const SwitchKey &key, int nb, int reps);
    Buf inner_product(const ModUp &m, const SwitchKey &key);
    // relinearisation tail: base (both components) + ModDown(acc), rescaled by q_l
    // with factor k and constant *cadd, into out at level l - 1
    void moddown_rescale_into(const Buf &acc, int l, int nb, const u64 *base, long base_ls, long base_es, long k,
                              const double *cadd, Ct &out);
    // batches of single ciphertexts at one level
    Ct pack(const std::vector<const Ct *> &cts);
    Ct unpack(const Ct &batch, int e);
    // rotations of one ciphertext by several steps sharing one ModUp
    std::vector<Ct> rotate_many(const Ct &a, const std::vector<long> &steps, const Keys &k);

    // plaintexts
    Buf encode_ntt(const double *z, size_t n, double scale, int nl, bool montgomery);
    Pt const_pt(double c, double scale, int nl);
    Pt vec_pt(const double *z, size_t n, double scale, int nl);
    // several slot-vector plaintexts at once: the host encodings run on
    // parallel threads, then each is uploaded and transformed
    std::vector<Pt> vec_pts(const std::vector<const std::vector<double> *> &zs, double scale, int nl,
                            const std::vector<const std::vector<double> *> *ims = nullptr);

    // tables
    const KsTable &ks_table(int l);
    const Buf &rescale_table(int l, long k = 1);
    const Buf &int_factor(long k);  // [2][L+1] k mod q_i and Shoup
    const u64 *rescale_addend(int l, long k, double c);
    const u64 *const_residues(double c, double scale);

    // client side
    void keygen(u64 seed, const std::vector<long> &steps, SecretKey *&sk, Keys *&ek);
    // the secret in NTT form over the first nl limbs of q_0..q_L, p_0.. (nl <= L+1+alpha),
    // on the device for one client operation
    Buf secret_ntt(const SecretKey &sk, int nl);
    void wipe(const Buf &b);  // zero a buffer that held secret material
    void gen_switch_key(const u64 *s_ntt, u64 seed, u32 key_id, const u64 *sp_ntt, SwitchKey &out);
    void key_fp(SwitchKey &k);
    Ct encrypt(const SecretKey &sk, const double *x, size_t n, u64 seed);
    void decrypt(const SecretKey &sk, const Ct &c, double *y, size_t n);
    // server side: evaluation keys from exported material (coefficient form,
    // [dnum][2][L+1+alpha][N] per key), and one digit of a key back out
    Keys *import_keys(const std::vector<u32> &ids, const std::vector<const u64 *> &data);
    void export_key(const Keys &k, u32 key_id, int digit, u64 *out);

    // transfers
    void upload(u64 *dst, const u64 *src, size_t words);
    void download(u64 *dst, const u64 *src, size_t words);
    void sync();
};

}  // namespace hk
