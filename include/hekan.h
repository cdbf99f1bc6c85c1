/*
 * hekan.h -- C ABI of the MI355X (gfx950) encrypted-KAN inference library.
 *
 * The library evaluates the privacy-preserving KAN inference of "Efficient
 * Privacy-Preserving KAN Inference Using Homomorphic Encryption" on one GPU:
 * RNS-CKKS ciphertext arithmetic (Preliminaries, Homomorphic Encryption: the
 * SIMD operations add, subtract, multiply and rotate) implemented as HIP
 * kernels, and the paper's evaluators on top of it (Method: SiLU
 * Approximation, B-spline Basis Approximation with Algorithms 1 and 2, Lazy
 * Combination and Fusion Linear Layer with Algorithm 3 and BSGS products).
 *
 * Roles follow the threat model of the paper (Preliminaries, Threat Model):
 * the client owns the secret key, encrypts the raster-scanned input and
 * decrypts the result; the server holds the plaintext model and the
 * evaluation keys and runs he_eval_kan without ever decrypting.
 *
 * Conventions for every function:
 *   - the return value is HE_OK (0) or a negative HE_E* code; no exception or
 *     C++ object crosses this boundary; he_last_error(ctx) returns a
 *     NUL-terminated message for the last failure on that context;
 *   - pointers to double/uint64_t/int32_t buffers are HOST pointers owned by
 *     the caller; the library copies what it needs before returning;
 *   - every handle (he_ctx, he_model, he_secret_key, he_eval_keys, he_ct,
 *     he_graph) is owned by the library and released with the matching
 *     *_free / he_ctx_destroy; handles keep their data resident in device
 *     memory (HBM), except the secret key, which stays in host memory;
 *   - handles may be released in any order: he_ctx_destroy ends the context
 *     for the caller at once (no further call may pass it), and the library
 *     releases its device memory when the last handle made from it is freed;
 *   - a handle passed together with a context must have been made by that
 *     context (HE_ESTATE otherwise);
 *   - a context is not thread-safe: use one context per host thread; work is
 *     issued on the context's stream and functions that return host data
 *     synchronise that stream;
 *   - slot vectors are real; slot j holds x[j] (raster order), the remaining
 *     slots of the N/2 are zero.
 */
#ifndef HEKAN_H
#define HEKAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HE_OK = 0,
    HE_EINVAL = -1,  /* bad argument (null pointer, size, out of range)         */
    HE_ENOMEM = -2,  /* host or device allocation failed, or buffer too small   */
    HE_EDEPTH = -3,  /* the circuit needs more levels than its operand has      */
    HE_ESHAPE = -4,  /* packing impossible: n_in (g+2k) slots exceed N/2       */
    HE_EKEY = -5,    /* a Galois key needed for a rotation was not generated    */
    HE_EDEVICE = -6, /* a HIP call or a kernel launch failed                    */
    HE_ESTATE = -7,  /* handle used with the wrong context or in a bad state    */
    HE_EAGAIN = -8   /* he_poll: the request has not finished yet               */
};

typedef struct he_ctx he_ctx;
typedef struct he_model he_model;
typedef struct he_secret_key he_secret_key;
typedef struct he_eval_keys he_eval_keys;
typedef struct he_ct he_ct;
typedef struct he_graph he_graph;
typedef struct he_server he_server;

/*
 * RNS-CKKS parameters (the paper's Experiment Setup fixes N = 2^16 with a
 * base prime, scale primes and special primes; the sizes here are inputs).
 * Primes are all 1 mod 2N: q_0 is the largest prime below 2^base_bits, the
 * special primes are the next ones below 2^special_bits, and q_L..q_1 are
 * chosen top-down as the prime nearest S_l^2 / 2^scale_bits, where S_L =
 * 2^scale_bits and S_{l-1} = S_l^2 / q_l is the canonical scale of level l-1.
 */
typedef struct {
    int32_t log_n;          /* ring degree N = 2^log_n, 10 <= log_n <= 16           */
    int32_t levels;         /* L: number of scale primes q_1..q_L                   */
    int32_t scale_bits;     /* Delta = 2^scale_bits (<= 58)                         */
    int32_t base_bits;      /* bits of q_0 (<= 60)                                  */
    int32_t special_count;  /* alpha: number of special primes (>= 1)               */
    int32_t special_bits;   /* bits of the special primes (<= 60)                   */
    int32_t digit_width;    /* Q limbs per hybrid key-switching digit, 1..8, with   */
                            /* ceil((levels + 1) / digit_width) <= 16 digits        */
    double sigma;           /* standard deviation of the rounded Gaussian error     */
    int32_t integer_words;  /* 0: primes below 2^46 run their transforms, basis     */
                            /* conversions and rescale tails in exact FP64          */
                            /* arithmetic, the others on 64-bit integer words; 1:  */
                            /* every prime on 64-bit integer words (Shoup, Barrett, */
                            /* Montgomery).  Both give the same residues.           */
    int32_t boot_levels;    /* levels kept for bootstrapping (0: none): the top     */
                            /* boot_levels primes have boot_bits bits and the       */
                            /* canonical scales there stay near 2^boot_bits (S_L =  */
                            /* 2^boot_bits); the computation levels below keep      */
                            /* scale_bits, their top level L_c = levels -           */
                            /* boot_levels with S = 2^scale_bits.  Fresh            */
                            /* encryptions and bootstrapping results are at L_c.    */
    int32_t boot_bits;      /* <= 58; digits must stay within the special primes'   */
                            /* product for the key-switch noise to stay small       */
    int32_t secret_hamming_weight; /* h > 0: the secret has exactly h non-zero      */
                            /* coefficients in {-1, 1} (sparse ternary, which keeps */
                            /* bootstrapping's overflow |I| small); 0: uniform      */
                            /* ternary                                              */
} he_params;

/*
 * One KANLayer n_in -> n_out with its HE-friendly constants (Method).
 * All arrays are row-major doubles owned by the caller.
 *   knots        g+2k+1 knots t_1..t_r (non-decreasing)
 *   wb, ws       n_out x n_in base weights and spline scales (phi = w_b b + w_s spline)
 *   c            n_out x n_in x (g+k) spline coefficients per edge
 *   silu_coeffs  Chebyshev series of the SiLU approximation on [silu_lo, silu_hi]
 *                (degree silu_degree, silu_degree+1 coefficients)
 *   comp_*       the comparison polynomial PolyComp as a composite of
 *                comp_stages odd polynomials; stage s has comp_stage_len[s]
 *                (2, 3 or 4) coefficients a_1, a_3, .. of odd powers, all
 *                stages concatenated in comp_coeffs; the final 1/2 is folded
 *                into the last stage and the evaluator adds 1/2 at the end.
 *   comp_prescale  if non-zero, the comparison inputs x - t are multiplied by
 *                this factor (1/(2R), Algorithm 2) in one rescale before the
 *                first stage; if zero the factor is folded into stage 0.
 */
typedef struct {
    int32_t n_in, n_out, g, k;
    const double *knots;
    const double *wb, *ws, *c;
    int32_t silu_degree;
    const double *silu_coeffs;
    double silu_lo, silu_hi;
    int32_t comp_stages;
    const int32_t *comp_stage_len;
    const double *comp_coeffs;
    double comp_prescale;
} he_kan_layer;

typedef struct {
    int32_t n_layers;
    const he_kan_layer *layers;
    /* input vectors per ciphertext, a power of two (0 reads as 1): feature i
     * of vector s in slot i S + s, output o of vector s in slot o S + s; the
     * linear layers act as W (x) I_S, whose only non-zero generalised
     * diagonals are multiples of S, so rotations are S times longer but as
     * many.  Every layer must fit: (g+2k) blocks of (previous output period
     * d) S slots within N/2. */
    int32_t samples_per_ct;
    /* Which restructurings of the paper's layer circuit to apply (a bitwise OR
     * of HE_CIRCUIT_*; 0 runs the circuit in the paper's order: Algorithm 2
     * with both PolyComps, W_f times the bases and W_b times the SiLU values
     * as two products, each folded over all slots).  None changes a value of
     * the FP64 circuit; each cuts key switches or their ModDowns. */
    int32_t circuit;
} he_kan_desc;

enum {
    /* The second comparison S((t_{m+2} - x)/2R) is 1 - S((x - t_{m+2})/2R)
     * because the composite is odd: 1 minus the first comparison of block
     * m+1 (one rotation instead of a second PolyComp), where the input holds
     * g+2k+1 blocks. */
    HE_CIRCUIT_SHARED_COMPARISON = 1,
    /* SiLU on the repeat-packed input, its coefficients masked to block g+k,
     * added to the bases: one product with [W_f | W_b] and one fold. */
    HE_CIRCUIT_FUSED_LINEAR = 2,
    /* A hidden layer's block layout repeats with the shortest power-of-two
     * period that holds its blocks; the fold runs over one period. */
    HE_CIRCUIT_FOLDED_PERIOD = 4,
    /* The giant-step rotations of each baby-step giant-step product share one
     * ModDown: their key-switch accumulators, each permuted by its
     * automorphism, are added over Q_l u P and divided by P once (Bossuat,
     * Mouchet, Troncoso-Pastoriza and Hubaux 2021).  Changes residues only by
     * the rounding of those divisions. */
    HE_CIRCUIT_SHARED_MODDOWN = 16,
    /* every restructuring */
    HE_CIRCUIT_RESTRUCTURED = 23,
    /* Not a restructuring: the comparison method of the paper's experiments
     * on the basis approximation, without lazy combination.  The bases are
     * moved from ColTile order into row order by a homomorphic permutation
     * (Algorithm 3's P applied to the ciphertext: one ciphertext-plaintext
     * product per distinct slot offset, baby-step giant-step rotations) and
     * multiplied by W' itself.  Costs one more level per layer; excludes
     * HE_CIRCUIT_FUSED_LINEAR and HE_CIRCUIT_FOLDED_PERIOD (HE_EINVAL). */
    HE_CIRCUIT_NAIVE_PERMUTATION = 8
};

/* ---------------------------------------------------------------- context */

/* Create a context: generates the prime chain and uploads NTT and
 * basis-conversion tables to the current HIP device.  hip_stream may be NULL
 * (the library creates its own stream) or a hipStream_t owned by the caller. */
int he_ctx_create(const he_params *p, void *hip_stream, he_ctx **out);
int he_ctx_destroy(he_ctx *ctx);
const char *he_last_error(const he_ctx *ctx);

/* Copy the primes q_0..q_L (levels+1 values), special primes (special_count
 * values) and canonical scales S_0..S_L (levels+1 values) to host arrays;
 * any pointer may be NULL. */
int he_ctx_primes(const he_ctx *ctx, uint64_t *q, uint64_t *p, double *scales);

/* Counters since creation: key switches, rescales, kernel launches. */
int he_ctx_counters(const he_ctx *ctx, uint64_t *keyswitches, uint64_t *rescales, uint64_t *launches);

/* Block until all work issued on the context's stream has completed. */
int he_ctx_sync(he_ctx *ctx);

/* Kernel timing for measurement: while enabled, every launch of one kernel
 * (0 forward NTT pass 1, 1 forward NTT pass 2, 2 inverse NTT pass 2,
 * 3 inverse NTT pass 1, 4 basis conversion, 5 key-switch inner product,
 * 6 ModUp's second pass fused with the key-switch inner product) is
 * bracketed by HIP events on the context stream.  kernel = -1 disables.
 * Enabling clears earlier records.  he_ctx_profile_read synchronises and
 * returns the summed event time, the number of launches, and the launches'
 * algorithmic bytes (every operand word read or written once) and operations
 * (NTT butterflies, or 64-bit multiply-accumulates). */
int he_ctx_profile(he_ctx *ctx, int32_t kernel);
int he_ctx_profile_read(he_ctx *ctx, double *total_ms, uint64_t *launches, double *bytes, double *ops);

/* Key-switch kernel configuration per (level, batch size): 0 = ModUp, then the
 * key inner product over every limb; 1, 8 or 32 = ModUp's second pass fused
 * with the inner product on the FP64 limbs, blocks ordered in spans of that
 * many (limb, row tile) groups (8, the default: the blocks of one group land
 * on one XCD whatever the batch element).  Every configuration computes the
 * same residues; only the time differs.
 * he_ctx_autotune times each configuration at every level 0..L for `batch`
 * elements (one key switch with the relinearisation key of ek on a zero input,
 * the median of `reps` runs after a warm-up), keeps the fastest for that batch
 * size, and writes the choices of levels 0..min(cap, L+1)-1 to choice and L+1
 * to *n.  It synchronises the stream (HE_ESTATE while a graph is being
 * captured on it).  he_ctx_set_keyswitch sets one entry by hand (HE_EINVAL for
 * another config value). */
int he_ctx_autotune(he_ctx *ctx, const he_eval_keys *ek, int32_t batch, int32_t reps, int32_t *choice, size_t cap,
                    size_t *n);
int he_ctx_set_keyswitch(he_ctx *ctx, int32_t level, int32_t batch, int32_t config);

/* Key-switch microbenchmark (measurement): `batch` ciphertexts at `level`
 * sharing one key, key-switched together `reps` times after one warm-up, each
 * repetition timed with HIP events on the context stream; writes the median
 * milliseconds of one repetition (one launch sequence for the whole batch).
 * step == 0 times the relinearisation of a ciphertext product as the library
 * runs it (key switch of d2 with ModDown and the following rescale in one
 * transform per limb; level >= 1); otherwise a rotation by `step` (automorphism
 * and key switch).  Operands are zero: the kernels' work does not depend on
 * the values.  Errors: HE_EKEY without the key, HE_EDEPTH for a product at
 * level 0, HE_EINVAL for other bad arguments. */
int he_ctx_bench_keyswitch(he_ctx *ctx, const he_eval_keys *ek, int32_t step, int32_t level, int32_t batch,
                           int32_t reps, double *ms);

/* ------------------------------------------------------------------ model */

/* Compile a KAN for encrypted evaluation: checks the layer shapes and their
 * packing (HE_ESHAPE), builds the fused weights W_f = W' P (Algorithm 3) and
 * records every rotation the circuit uses.  The level budget is checked when
 * a layer is evaluated: an input whose level cannot hold the layer's circuit
 * makes the evaluation return HE_EDEPTH (the step that would go below level
 * 0 stops it; no ciphertext below level 0 is ever formed).
 * If refresh_between_layers is non-zero each layer starts at the top level
 * (the caller refreshes the ciphertext between layers with he_eval_kan_layer). */
int he_model_compile(he_ctx *ctx, const he_kan_desc *desc, int32_t refresh_between_layers,
                     he_model **out);
int he_model_free(he_model *m);

/* Rotation steps (left shifts; negative = right) the model needs keys for.
 * Writes min(cap, total) steps and the total count to *n. */
int he_model_rotation_steps(const he_model *m, int32_t *steps, size_t cap, size_t *n);

/* Input layout (what the client encrypts).  The first layer's repeat packing
 * (Algorithm 1) needs n_in * 2^ceil(log2(g+2k)) slots; when that exceeds N/2
 * the input is split into chunks of consecutive features, each holding
 * cap = (N/2) / 2^ceil(log2(g+2k)) features and the last one the rest:
 * chunk c = features [c cap, min((c+1) cap, n_in)), encrypted as its own
 * ciphertext in slots [0, chunk size).  Writes the nc + 1 bounds
 * (min(cap, nc + 1) of them) and nc to *n_chunks. */
int he_model_input_chunks(const he_model *m, int32_t *bounds, size_t cap, size_t *n_chunks);
/* The period of layer `layer`'s output slots (d S: d the next power of two
 * >= the layer's n_out, S the vectors per ciphertext): the output repeats
 * with it over all N/2 slots, so a sparsely packed refresh of any multiple of
 * it keeps the output (he_boot_desc.slots).  HE_EINVAL for a layer out of
 * range. */
int he_model_output_period(const he_model *m, int32_t layer, int64_t *period);

/* -------------------------------------------------------------------- keys */

/* The secret key and the evaluation keys are separate handles, as the
 * paper's threat model separates the parties (Preliminaries, Threat Model):
 * the client keeps the secret key, the server evaluates with the evaluation
 * keys alone and never holds the secret.
 *
 * he_keygen draws a ternary secret s (kept in host memory inside *sk; a
 * client operation uploads it to the device for its own duration and clears
 * that copy before returning) and the evaluation keys resident in HBM (*ek):
 * the relinearisation key (for s^2) and one Galois key per rotation step in
 * steps[0..nsteps) (for sigma_{5^t}(s); HE_STEP_CONJUGATE for the complex
 * conjugation sigma_{2N-1}(s)).  The secret is uniform ternary, or sparse
 * ternary of the context's secret_hamming_weight.  All randomness is drawn
 * from ChaCha20 keyed by `seed`. */
int he_keygen(he_ctx *ctx, uint64_t seed, const int32_t *steps, size_t nsteps, he_secret_key **sk,
              he_eval_keys **ek);
int he_secret_key_free(he_secret_key *sk);
int he_eval_keys_free(he_eval_keys *ek);

/* Key ids held by ek: 0 for the relinearisation key, then the Galois elements
 * 5^t mod 2N in increasing order.  Writes min(cap, total) ids and the total
 * to *n. */
int he_eval_keys_ids(const he_eval_keys *ek, uint32_t *ids, size_t cap, size_t *n);

/* Export one digit of one switching key in coefficient form (what a client
 * sends to a server): key_id as in he_eval_keys_ids; writes the [2][L+1+alpha][N]
 * residues (b then a) of digit `digit` (0 <= digit < ceil((L+1) / digit_width)). */
int he_eval_keys_export(he_ctx *ctx, const he_eval_keys *ek, uint32_t key_id, int32_t digit, uint64_t *out,
                        size_t cap);

/* Build evaluation keys from exported key material alone (no secret): keys
 * ids[0..nkeys) (distinct, each 0 or a Galois element), key i given by
 * data[i] as [dnum][2][L+1+alpha][N] residues in coefficient form, digit
 * after digit as he_eval_keys_export writes them.  HE_EINVAL for an id that
 * is not a Galois element, a repeated id or an unreduced residue. */
int he_eval_keys_import(he_ctx *ctx, const uint32_t *ids, size_t nkeys, const uint64_t *const *data,
                        he_eval_keys **out);

/* ------------------------------------------------------------- ciphertexts */

/* Encrypt x[0..n) (raster-scanned input, slots n..N/2-1 are zero) under the
 * secret key at the top computation level L_c (levels - boot_levels):
 * (-a s + e + m, a), with a and e drawn from ChaCha20 keyed by `seed`. */
int he_encrypt(he_ctx *ctx, const he_secret_key *sk, const double *x, size_t n, uint64_t seed, he_ct **out);

/* Decrypt and decode the first n slots into y. */
int he_decrypt(he_ctx *ctx, const he_secret_key *sk, const he_ct *ct, double *y, size_t n);

/* Level of a ciphertext (its scale is the canonical S_level). */
int he_ct_level(const he_ct *ct);
int he_ct_free(he_ct *ct);

/* Export a ciphertext in coefficient form: [2][level+1][N] residues. */
int he_ct_export(he_ctx *ctx, const he_ct *ct, uint64_t *out, size_t cap);

/* Import a ciphertext given in coefficient form [2][level+1][N]. */
int he_ct_import(he_ctx *ctx, const uint64_t *in, int32_t level, he_ct **out);

/* ------------------------------------------------------------ bootstrapping */

/* The rotation "step" naming the complex conjugation (Galois element 2N - 1):
 * he_keygen makes its key when steps holds it; he_boot_rotation_steps lists it. */
#define HE_STEP_CONJUGATE INT32_MIN

/*
 * CKKS bootstrapping, the refresh the paper relies on (Experiments,
 * Experiment Setup: multiplicative depth 20 with bootstrapping in the
 * settings of Lee et al. 2022; the paper does not restate the procedure).
 * The library runs the full-slot RNS-CKKS bootstrapping on a context with
 * boot_levels > 0:
 *   ModRaise (the level-0 residues as centred integers, lifted to level L),
 *   CoeffToSlot (the inverse of the encoding's special DFT, its butterfly
 *     stages merged into cts_levels groups, each one baby-step giant-step
 *     product with the group's diagonals: one level each),
 *   the real/imaginary split by conjugation,
 *   EvalMod on both halves (the Chebyshev series cos_coeffs of
 *     cos(2 pi (y - 1/4) / 2^double_angles) on [-k_range, k_range], then
 *     double_angles steps c <- 2 c^2 - 1, giving sin(2 pi y)),
 *   SlotToCoeff (the special DFT in stc_levels groups, the last landing at
 *     the top computation level L_c).
 * k_range must bound |I| + 1/2, where the ModRaise plaintext is m + q_0 I
 * (|I| <= (h + 1) / 2 for a sparse secret of weight h; in practice a few
 * standard deviations of sqrt((h + 1) / 12)).  The levels used are
 * cts_levels + the series' depth + double_angles + stc_levels and must fit
 * in boot_levels (HE_EDEPTH at evaluation otherwise).
 */
typedef struct {
    int32_t cts_levels;        /* 1 .. log_n - 1 (log2 slots when sparse) */
    int32_t stc_levels;        /* 1 .. log_n - 1 (log2 slots when sparse) */
    double k_range;            /* K > 0 */
    int32_t double_angles;     /* r >= 0 */
    int32_t cos_degree;        /* >= 1 */
    const double *cos_coeffs;  /* cos_degree + 1 Chebyshev coefficients */
    /* 0: the full-slot refresh above (complex slot values kept).  1: real slot
     * values, SlotToCoeff first (Chen, Chillotti, Song 2019): the special DFT
     * runs on the input's own limbs (the input must be at level >= stc_levels;
     * it puts the slots, times 2^-7, into the low coefficients), then ModRaise,
     * CoeffToSlot, the real half w + conj(w) through one EvalMod, and one
     * product by q_0 / (2 pi S 2^-7) (S the scale after SlotToCoeff) landing at
     * L_c.  The result holds the real parts of the slots; it uses
     * cts_levels + the series' depth + double_angles + 1 boot levels. */
    int32_t real_slots;
    /* 0: all N/2 slots.  Else n, a power of two from 2 to N/2: a sparsely
     * packed refresh (Cheon, Han, Kim, Kim, Song 2018) of a message whose slot
     * vector repeats with period n (a polynomial in X^(N/(2n))): after ModRaise
     * SubSum adds the rotations by n 2^k (k < log2(N/(2n))), and CoeffToSlot
     * and SlotToCoeff run only the first log2 n butterfly stages (which act
     * on every aligned block of n slots as the n-slot special DFT), so
     * cts_levels and stc_levels are at most log2 n.  With real_slots = 1 the
     * SlotToCoeff that runs first is sparse as well. */
    int32_t slots;
} he_boot_desc;

typedef struct he_boot he_boot;

/* Build the bootstrapping plan (the merged diagonals of every stage group;
 * their plaintexts are encoded on first use and kept in HBM with the plan
 * until he_boot_free; SlotToCoeff's first group carries the input's scale, so
 * its plaintexts are kept once per input level used). */
int he_boot_create(he_ctx *ctx, const he_boot_desc *desc, he_boot **out);
int he_boot_free(he_boot *b);

/* Rotation steps the bootstrapping needs keys for, HE_STEP_CONJUGATE
 * included.  Writes min(cap, total) steps and the total to *n. */
int he_boot_rotation_steps(const he_boot *b, int32_t *steps, size_t cap, size_t *n);

/* Refresh in (at a computation level <= L_c, values with |m| well below
 * q_0 / 2): *out is a new ciphertext at L_c with the same slot values (up to
 * the approximation error).  Asynchronous on the context stream.  Errors:
 * HE_EKEY without a needed key, HE_EDEPTH if the plan does not fit the boot
 * levels, HE_EINVAL for an input above L_c. */
int he_bootstrap(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *in, he_ct **out);

/* The same for n ciphertexts at one level in one batched pass (every ring
 * kernel covers all of them); out receives n ciphertexts. */
int he_bootstrap_batch(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *const *in, size_t n,
                       he_ct **out);

/* The network on n requests (as he_eval_kan_batch: in holds n * nc input
 * chunks, request-major) with a bootstrapping of every layer's output before
 * the next layer, in place of the client-aided refresh: the whole inference
 * runs on the server.  Each layer must fit the computation levels (HE_EDEPTH
 * otherwise); the model is compiled with refresh_between_layers = 1.  A
 * sparsely packed plan's slots must be a multiple of every refreshed layer's
 * output period (he_model_output_period; HE_ESHAPE otherwise). */
int he_eval_kan_boot(he_ctx *ctx, const he_model *m, he_boot *b, const he_eval_keys *ek, const he_ct *const *in,
                     size_t n, he_ct **out);

/* The stages of he_bootstrap, each as it runs there:
 *   he_boot_coeff_to_slot: ModRaise of in (taken at level 0) and CoeffToSlot,
 *     the result at level L - cts_levels holding (t_k + i t_{k+N/2}) / (2 q_0)
 *     in bit-reversed slot order k;
 *   he_boot_eval_mod: EvalMod of in (slots in [-k_range, k_range]);
 *   he_boot_slot_to_coeff: SlotToCoeff of in for a bootstrapping input that
 *     was at source_level (its scale enters SlotToCoeff's constant), the
 *     result at L_c.
 * he_bootstrap splits the first result w into w + conj(w) and
 * i (conj(w) - w) (he_ct_rotate with HE_STEP_CONJUGATE, he_ct_mul_i), runs
 * both through EvalMod as one batch and recombines u_0 + i u_1. */
int he_boot_coeff_to_slot(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *in, he_ct **out);
int he_boot_eval_mod(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *in, he_ct **out);
int he_boot_slot_to_coeff(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *in, int32_t source_level,
                          he_ct **out);

/* ------------------------------------------------------- encrypted inference */

/* Run the whole network on `in` (server side; no secret key involved) for a
 * model with one input ciphertext (HE_ESHAPE otherwise).  Asynchronous on the
 * context stream; *out is a new ciphertext. */
int he_eval_kan(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, const he_ct *in, he_ct **out);

/* The same for any input layout: in[0..n_in) are the input chunks in order
 * (n_in must equal he_model_input_chunks' count, HE_ESHAPE otherwise).  Each
 * chunk runs the first layer's packing, bases and SiLU on its own and is
 * multiplied by its columns of the layer's weights; the partial sums are
 * added before the layer's fold. */
int he_eval_kan_chunks(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, const he_ct *const *in, size_t n_in,
                       he_ct **out);

/* Run layer `layer` only (for client-aided refresh between layers); layer 0
 * of a model with several input chunks needs he_eval_kan_layer_batch. */
int he_eval_kan_layer(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, int32_t layer, const he_ct *in,
                      he_ct **out);

/* Run the network on n independent requests in one batched pass: every ring
 * kernel processes all requests' limbs in one launch.  in holds n * nc
 * ciphertexts, request-major (request i's chunk c at in[i nc + c], nc = the
 * model's input chunk count); out receives n ciphertexts. */
int he_eval_kan_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, const he_ct *const *in, size_t n,
                      he_ct **out);

/* A batched inference (as he_eval_kan_batch) captured once into a HIP graph
 * and replayed: the schedule of one layer after another, for callers that
 * evaluate the same request set repeatedly (and to take the host's launch
 * cost off the device's critical path).  The call runs the inference once
 * eagerly (filling every cache, so the captured run makes no host transfer or
 * synchronisation) and then captures a second run on the context stream; out
 * receives n ciphertexts holding its result.  Each he_graph_launch recomputes
 * them in place, asynchronously on the context stream, from the current
 * contents of the same input ciphertexts.  The graph keeps its inputs,
 * outputs and temporaries allocated until he_graph_free (freeing the handles
 * earlier is allowed); free it before its context.  Errors: HE_EINVAL for
 * null arguments or n = 0, HE_EDEVICE if the runtime refuses the capture. */
int he_graph_capture_kan_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, const he_ct *const *in, size_t n,
                               he_ct **out, he_graph **g);
int he_graph_launch(he_graph *g);
int he_graph_free(he_graph *g);

/* A bootstrapping of n ciphertexts at one level (as he_bootstrap_batch)
 * captured the same way: one eager run, then a captured run; out receives n
 * ciphertexts, which each he_graph_launch recomputes in place from the
 * current contents of the inputs.  Same errors as he_graph_capture_kan_batch
 * plus those of he_bootstrap. */
int he_graph_capture_bootstrap(he_ctx *ctx, he_boot *b, const he_eval_keys *ek, const he_ct *const *in, size_t n,
                               he_ct **out, he_graph **g);

/* Run layer `layer` on n requests (all at the same level) in one batched
 * pass: the building block of layer-granular continuous batching.  For layer
 * 0, in holds n * nc ciphertexts laid out as for he_eval_kan_batch; for later
 * layers, n. */
int he_eval_kan_layer_batch(he_ctx *ctx, const he_model *m, const he_eval_keys *ek, int32_t layer,
                            const he_ct *const *in, size_t n, he_ct **out);

/* Native continuous batching (a project addition; the paper evaluates one
 * request at a time).  A server owns a worker thread that runs submitted
 * requests layer by layer on the context's stream: it admits them in
 * submission order while their models' working memory fits hbm_budget bytes
 * (a model's first request runs alone, and its peak pool growth is taken as
 * the model's working memory; the pool's peak counter is reset for that),
 * then repeatedly evaluates the (model, layer) group of the oldest admitted
 * request as one batch of up to max_batch requests, so requests submitted
 * while others run share launches with them.  While a server exists no other
 * thread may issue work on its context (he_submit and he_poll may be called
 * from any thread).  he_submit queues one request (in[0..n_in): its input
 * chunks as for he_eval_kan_chunks, single ciphertexts of the server's
 * context at one level; the server keeps its own reference, so the caller may
 * free them) and writes its tag.  he_poll returns HE_OK with the request's
 * output in *out (a new ciphertext) and the time from submission to
 * completion in *latency_ms (may be NULL), HE_EAGAIN if it has not finished
 * within wait_ms milliseconds (0: do not wait), the error code of the failed
 * evaluation, or HE_EINVAL for a tag that is not pending (never submitted or
 * already taken).  he_server_stats: requests finished, layer batches run and
 * the requests they held (mean batch = runs / batches).  he_server_destroy
 * finishes every submitted request, frees the results not taken, and joins
 * the worker. */
int he_server_create(he_ctx *ctx, const he_eval_keys *ek, int32_t max_batch, uint64_t hbm_budget, he_server **out);
int he_submit(he_server *s, const he_model *m, const he_ct *const *in, size_t n_in, uint64_t *tag);
int he_poll(he_server *s, uint64_t tag, int32_t wait_ms, he_ct **out, double *latency_ms);
int he_server_stats(he_server *s, uint64_t *completed, uint64_t *layer_batches, uint64_t *layer_runs);
int he_server_destroy(he_server *s);

/* Device memory held by the context's pool: bytes in live buffers, bytes
 * cached for reuse, and the peak of live bytes since the last reset
 * (reset_peak != 0 resets it to the current live bytes). */
int he_ctx_memory(he_ctx *ctx, uint64_t *live, uint64_t *cached, uint64_t *peak, int32_t reset_peak);

/* Free and total device memory of the context's device as the runtime
 * reports them (hipMemGetInfo); the bytes the context's pool caches count as
 * used.  For admission budgets. */
int he_ctx_device_memory(he_ctx *ctx, uint64_t *free_bytes, uint64_t *total_bytes);

/* ------------------------------------------------ individual homomorphic ops */

/* out = a + b (same level). */
int he_ct_add(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
/* out = a - b (same level). */
int he_ct_sub(he_ctx *ctx, const he_ct *a, const he_ct *b, he_ct **out);
/* out = a with its limbs above `level` dropped (0 <= level <= a's level): the
 * same plaintext, read at the canonical scale of the lower level. */
int he_ct_mod_drop(he_ctx *ctx, const he_ct *a, int32_t level, he_ct **out);
/* out = a X^(N/2): every slot times i (zeta^(5^j N/2) = i); exact, no level. */
int he_ct_mul_i(he_ctx *ctx, const he_ct *a, he_ct **out);
/* ModRaise (bootstrapping's first step): a at level 0, its residues mod q_0
 * read as centred integers and lifted to every prime of level L. */
int he_ct_mod_raise(he_ctx *ctx, const he_ct *a, he_ct **out);
/* out = a (x) b: tensor, relinearise (hybrid key switch), rescale (level - 1). */
int he_ct_mul(he_ctx *ctx, const he_eval_keys *ek, const he_ct *a, const he_ct *b, he_ct **out);
/* out = rot(a, step): slots move left by step (right if negative). */
int he_ct_rotate(he_ctx *ctx, const he_eval_keys *ek, const he_ct *a, int32_t step, he_ct **out);
/* out = sum_i rot(in[i], steps[i]) for n >= 1 ciphertexts of one level and
 * batch size (steps[i] = 0: the term is added as it is) with a single
 * ModDown: each rotation's key-switch accumulators over Q_l u P, permuted by
 * its automorphism, plus P times its permuted c_0, are added and divided by P
 * once (the giant steps of a baby-step giant-step product; Bossuat, Mouchet,
 * Troncoso-Pastoriza and Hubaux 2021).  The residues differ from those of n
 * separate he_ct_rotate calls added up only by the rounding of the divisions
 * by P.  HE_ESHAPE if the levels or batch sizes differ, HE_EKEY if a step has
 * no key. */
int he_ct_rotate_sum(he_ctx *ctx, const he_eval_keys *ek, const he_ct *const *in, const int32_t *steps, size_t n,
                     he_ct **out);
/* out = rescale(a): divide by q_level with rounding, drop one limb. */
int he_ct_rescale(he_ctx *ctx, const he_ct *a, he_ct **out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): he_ct_rescale into an
 * existing ciphertext, calling no allocator.  out must be a ciphertext of the
 * same context at level a.level - 1 (a result of an earlier call, or
 * he_ct_import); its residues are overwritten with rescale(a), the same
 * residues he_ct_rescale returns.  The staging between the rescale's passes
 * lives in a device array of 32 MiB that the library holds on every device it
 * runs on until the process ends, shared by all contexts there: a rescale
 * needs (level + 1) 2 N 8 bytes of it, and a larger one returns HE_ENOMEM
 * with nothing launched (at N = 2^16 up to level 31).  Calls that overlap
 * on one device race for that array.  Errors: HE_EINVAL (null, batched,
 * wrong output level, output sharing memory with a or with any other
 * ciphertext or graph), HE_EDEPTH (a at level 0), HE_ESTATE (handles of
 * another context). */
int he_ct_rescale_noalloc(he_ctx *ctx, const he_ct *a, he_ct *out);

/* out = sum_i a[i] * z_i landing at level `target` with scale S_target; z_i
 * is the slot vector z + i*slots (n_slots values each) or, when n_slots == 1,
 * the constant z[i]. */
int he_ct_lincomb(he_ctx *ctx, const he_ct *const *a, size_t n, const double *z, size_t n_slots,
                  int32_t target, he_ct **out);

/* Negacyclic product of two polynomials given in coefficient form over the
 * first nl limbs of the chain (q_0..): NTT, pointwise product, inverse NTT on
 * the GPU.  a, b, out: [nl][N] residues. */
int he_poly_mul(he_ctx *ctx, const uint64_t *a, const uint64_t *b, int32_t nl, uint64_t *out);

/* Encode slot values at `scale` into residues over nl limbs (coefficient
 * form): round(scale * tau^-1(z)) with ties to even. */
int he_encode(he_ctx *ctx, const double *z, size_t n, double scale, int32_t nl, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
