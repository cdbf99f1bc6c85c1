"""Thin ctypes binding of libhekan.so (include/hekan.h).  Argument marshalling
only: every homomorphic operation runs in the library's HIP kernels.  There is
no CPU fallback; if the library is missing this module raises on import of
the library (call `python -m paper_2409_07751_amd.build` first)."""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhekan.so")

HE_OK, HE_EINVAL, HE_ENOMEM, HE_EDEPTH, HE_ESHAPE, HE_EKEY, HE_EDEVICE, HE_ESTATE, HE_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
_NAMES = {-1: "HE_EINVAL", -2: "HE_ENOMEM", -3: "HE_EDEPTH", -4: "HE_ESHAPE", -5: "HE_EKEY", -6: "HE_EDEVICE",
          -7: "HE_ESTATE", -8: "HE_EAGAIN"}


class HeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class he_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int32), ("levels", ctypes.c_int32), ("scale_bits", ctypes.c_int32),
                ("base_bits", ctypes.c_int32), ("special_count", ctypes.c_int32),
                ("special_bits", ctypes.c_int32), ("digit_width", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("integer_words", ctypes.c_int32), ("boot_levels", ctypes.c_int32), ("boot_bits", ctypes.c_int32),
                ("secret_hamming_weight", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class he_kan_layer(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_out", ctypes.c_int32), ("g", ctypes.c_int32), ("k", ctypes.c_int32),
                ("knots", _dp), ("wb", _dp), ("ws", _dp), ("c", _dp), ("silu_degree", ctypes.c_int32),
                ("silu_coeffs", _dp), ("silu_lo", ctypes.c_double), ("silu_hi", ctypes.c_double),
                ("comp_stages", ctypes.c_int32), ("comp_stage_len", _i32p), ("comp_coeffs", _dp),
                ("comp_prescale", ctypes.c_double)]


class he_kan_desc(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("layers", ctypes.POINTER(he_kan_layer)),
                ("samples_per_ct", ctypes.c_int32), ("circuit", ctypes.c_int32)]


class he_boot_desc(ctypes.Structure):
    _fields_ = [("cts_levels", ctypes.c_int32), ("stc_levels", ctypes.c_int32), ("k_range", ctypes.c_double),
                ("double_angles", ctypes.c_int32), ("cos_degree", ctypes.c_int32), ("cos_coeffs", _dp),
                ("real_slots", ctypes.c_int32), ("slots", ctypes.c_int32)]


# the rotation "step" naming the complex conjugation (HE_STEP_CONJUGATE)
STEP_CONJUGATE = -(1 << 31)

# he_kan_desc.circuit: restructurings of the paper's layer circuit (0 = the paper's order)
CIRCUIT_PAPER = 0
CIRCUIT_SHARED_COMPARISON, CIRCUIT_FUSED_LINEAR, CIRCUIT_FOLDED_PERIOD = 1, 2, 4
CIRCUIT_SHARED_MODDOWN = 16
CIRCUIT_RESTRUCTURED = 23
CIRCUIT_NAIVE_PERMUTATION = 8


_lib = None

_SIGS = {
    "he_ctx_create": [ctypes.POINTER(he_params), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_ctx_destroy": [ctypes.c_void_p],
    "he_ctx_primes": [ctypes.c_void_p, _u64p, _u64p, _dp],
    "he_ctx_counters": [ctypes.c_void_p, _u64p, _u64p, _u64p],
    "he_ctx_sync": [ctypes.c_void_p],
    "he_ctx_profile": [ctypes.c_void_p, ctypes.c_int32],
    "he_ctx_autotune": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                        ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "he_ctx_set_keyswitch": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "he_ctx_bench_keyswitch": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, _dp],
    "he_graph_capture_kan_batch": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p],
    "he_graph_capture_bootstrap": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p],
    "he_graph_launch": [ctypes.c_void_p],
    "he_graph_free": [ctypes.c_void_p],
    "he_ctx_profile_read": [ctypes.c_void_p, _dp, _u64p, _dp, _dp],
    "he_model_compile": [ctypes.c_void_p, ctypes.POINTER(he_kan_desc), ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_void_p)],
    "he_model_free": [ctypes.c_void_p],
    "he_boot_create": [ctypes.c_void_p, ctypes.POINTER(he_boot_desc), ctypes.POINTER(ctypes.c_void_p)],
    "he_boot_free": [ctypes.c_void_p],
    "he_boot_rotation_steps": [ctypes.c_void_p, _i32p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "he_bootstrap": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.POINTER(ctypes.c_void_p)],
    "he_boot_coeff_to_slot": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_void_p)],
    "he_boot_eval_mod": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.POINTER(ctypes.c_void_p)],
    "he_boot_slot_to_coeff": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan_boot": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_sub": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_mul_i": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_mod_drop": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_mod_raise": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_bootstrap_batch": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                           ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_model_rotation_steps": [ctypes.c_void_p, _i32p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "he_model_input_chunks": [ctypes.c_void_p, _i32p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "he_model_output_period": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)],
    "he_keygen": [ctypes.c_void_p, ctypes.c_uint64, _i32p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p),
                  ctypes.POINTER(ctypes.c_void_p)],
    "he_secret_key_free": [ctypes.c_void_p],
    "he_eval_keys_free": [ctypes.c_void_p],
    "he_eval_keys_ids": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_size_t,
                         ctypes.POINTER(ctypes.c_size_t)],
    "he_eval_keys_export": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, _u64p,
                            ctypes.c_size_t],
    "he_eval_keys_import": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_size_t,
                            ctypes.POINTER(_u64p), ctypes.POINTER(ctypes.c_void_p)],
    "he_encrypt": [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_size_t, ctypes.c_uint64,
                   ctypes.POINTER(ctypes.c_void_p)],
    "he_decrypt": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_size_t],
    "he_ct_level": [ctypes.c_void_p],
    "he_ct_free": [ctypes.c_void_p],
    "he_ct_export": [ctypes.c_void_p, ctypes.c_void_p, _u64p, ctypes.c_size_t],
    "he_ct_import": [ctypes.c_void_p, _u64p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan_chunks": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                           ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan_layer": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan_batch": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                          ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_eval_kan_layer_batch": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_ctx_memory": [ctypes.c_void_p, _u64p, _u64p, _u64p, ctypes.c_int32],
    "he_server_create": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                         ctypes.POINTER(ctypes.c_void_p)],
    "he_submit": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t,
                  ctypes.POINTER(ctypes.c_uint64)],
    "he_poll": [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), _dp],
    "he_server_stats": [ctypes.c_void_p, _u64p, _u64p, _u64p],
    "he_server_destroy": [ctypes.c_void_p],
    "he_ctx_device_memory": [ctypes.c_void_p, _u64p, _u64p],
    "he_ct_add": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_mul": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_rotate": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                     ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_rotate_sum": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                         ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_rescale": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)],
    "he_ct_rescale_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "he_ct_lincomb": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t, _dp, ctypes.c_size_t,
                      ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)],
    "he_poly_mul": [ctypes.c_void_p, _u64p, _u64p, ctypes.c_int32, _u64p],
    "he_encode": [ctypes.c_void_p, _dp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int32, _u64p],
}


def lib():
    """Load libhekan.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhekan.so is not built; run `python -m paper_2409_07751_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.he_last_error.argtypes = [ctypes.c_void_p]
        L.he_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a):
    t = {np.float64: _dp, np.int32: _i32p, np.uint64: _u64p}[a.dtype.type]
    return a.ctypes.data_as(t)


class Context:
    """RNS-CKKS context on the current HIP device (see he_params)."""

    def __init__(self, log_n, levels, scale_bits, special_count, digit_width, base_bits=60, special_bits=60,
                 sigma=3.2, stream=None, integer_words=False, boot_levels=0, boot_bits=0, hamming_weight=0):
        self.lib = lib()
        p = he_params(log_n, levels, scale_bits, base_bits, special_count, special_bits, digit_width, sigma,
                      1 if integer_words else 0, boot_levels, boot_bits, hamming_weight)
        h = ctypes.c_void_p()
        rc = self.lib.he_ctx_create(ctypes.byref(p), ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if rc != HE_OK:
            raise HeError(rc, "context creation failed")
        self.h = h
        self.log_n, self.N, self.L, self.alpha, self.w = log_n, 1 << log_n, levels, special_count, digit_width
        self.slots = self.N // 2
        self.top = levels - boot_levels  # top computation level

    def check(self, rc):
        if rc != HE_OK:
            raise HeError(rc, self.lib.he_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.he_ctx_destroy(self.h)
            self.h = None

    def primes(self):
        q = np.zeros(self.L + 1, np.uint64)
        p = np.zeros(self.alpha, np.uint64)
        S = np.zeros(self.L + 1, np.float64)
        self.check(self.lib.he_ctx_primes(self.h, _ptr(q), _ptr(p), _ptr(S)))
        return q, p, S

    def counters(self):
        v = [ctypes.c_uint64() for _ in range(3)]
        self.check(self.lib.he_ctx_counters(self.h, *[ctypes.byref(x) for x in v]))
        return {"keyswitches": v[0].value, "rescales": v[1].value, "launches": v[2].value}

    def sync(self):
        self.check(self.lib.he_ctx_sync(self.h))

    KERNELS = {"ntt_fwd_pass1": 0, "ntt_fwd_pass2": 1, "ntt_inv_pass2": 2, "ntt_inv_pass1": 3, "bconv": 4,
               "keyip": 5, "modup_keyip": 6}

    def autotune(self, keys, batch, reps=3):
        """he_ctx_autotune: the key-switch configuration chosen at each level
        0..L for this batch size (0 unfused; 1, 8, 32 fused with that span)."""
        choice = (ctypes.c_int32 * (self.L + 1))()
        n = ctypes.c_size_t()
        self.check(self.lib.he_ctx_autotune(self.h, _ek(keys), batch, reps, choice, self.L + 1, ctypes.byref(n)))
        return [int(choice[i]) for i in range(n.value)]

    def bench_keyswitch(self, keys, step, level, batch, reps=5):
        """he_ctx_bench_keyswitch: median ms of one key switch of `batch`
        ciphertexts at `level` (step 0: relinearisation with its rescale;
        otherwise a rotation by `step`)."""
        ms = ctypes.c_double()
        self.check(self.lib.he_ctx_bench_keyswitch(self.h, _ek(keys), step, level, batch, reps, ctypes.byref(ms)))
        return ms.value

    def set_keyswitch(self, level, batch, config):
        self.check(self.lib.he_ctx_set_keyswitch(self.h, level, batch, config))

    def profile(self, kernel):
        """Time every launch of `kernel` (a KERNELS name, or None to stop)."""
        self.check(self.lib.he_ctx_profile(self.h, -1 if kernel is None else self.KERNELS[kernel]))

    def profile_read(self):
        ms, by, ops = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_uint64()
        self.check(self.lib.he_ctx_profile_read(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
                                                ctypes.byref(ops)))
        return {"ms": ms.value, "launches": n.value, "bytes": by.value, "ops": ops.value}

    # -- keys, ciphertexts --------------------------------------------------
    def keygen(self, seed, steps):
        """he_keygen: a client's key pair (Keys: .sk the secret key, .ek the
        evaluation keys); calls below take the handle their role needs."""
        s = _arr(list(steps), np.int32)
        sk, ek = ctypes.c_void_p(), ctypes.c_void_p()
        self.check(self.lib.he_keygen(self.h, seed, _ptr(s) if len(s) else None, len(s), ctypes.byref(sk),
                                      ctypes.byref(ek)))
        return Keys(SecretKey(self, sk), EvalKeys(self, ek))

    def import_eval_keys(self, material):
        """he_eval_keys_import: evaluation keys from exported material alone
        ({key id: [dnum][2][L+1+alpha][N] residues}, e.g. EvalKeys.export_all())."""
        ids = sorted(material)
        arrs = [_arr(material[i], np.uint64) for i in ids]
        idv = (ctypes.c_uint32 * len(ids))(*ids)
        ptrs = (_u64p * len(ids))(*[_ptr(a) for a in arrs])
        h = ctypes.c_void_p()
        self.check(self.lib.he_eval_keys_import(self.h, idv, len(ids), ptrs, ctypes.byref(h)))
        return EvalKeys(self, h)

    def encrypt(self, keys, x, seed):
        x = _arr(x, np.float64)
        h = ctypes.c_void_p()
        self.check(self.lib.he_encrypt(self.h, _sk(keys), _ptr(x), len(x), seed, ctypes.byref(h)))
        return Ciphertext(self, h)

    def decrypt(self, keys, ct, n):
        y = np.zeros(n, np.float64)
        self.check(self.lib.he_decrypt(self.h, _sk(keys), ct.h, _ptr(y), n))
        return y

    def import_ct(self, res, level):
        res = _arr(res, np.uint64)
        assert res.shape == (2, level + 1, self.N)
        h = ctypes.c_void_p()
        self.check(self.lib.he_ct_import(self.h, _ptr(res), level, ctypes.byref(h)))
        return Ciphertext(self, h)

    def _new(self, fn, *args):
        h = ctypes.c_void_p()
        self.check(fn(self.h, *args, ctypes.byref(h)))
        return Ciphertext(self, h)

    def add(self, a, b):
        return self._new(self.lib.he_ct_add, a.h, b.h)

    def mul(self, keys, a, b):
        return self._new(self.lib.he_ct_mul, _ek(keys), a.h, b.h)

    def rotate(self, keys, a, step):
        return self._new(self.lib.he_ct_rotate, _ek(keys), a.h, step)

    def rotate_sum(self, keys, cts, steps):
        """he_ct_rotate_sum: sum_i rot(cts[i], steps[i]) with one ModDown."""
        if len(cts) != len(steps):
            raise ValueError("one step per ciphertext")
        hs = (ctypes.c_void_p * len(cts))(*[c.h.value for c in cts])
        st = (ctypes.c_int32 * len(steps))(*[int(s) for s in steps])
        return self._new(self.lib.he_ct_rotate_sum, _ek(keys), hs, st, len(cts))

    def rescale(self, a):
        return self._new(self.lib.he_ct_rescale, a.h)

    def rescale_noalloc(self, a, out):
        """he_ct_rescale_noalloc: rescale(a) written into the existing
        ciphertext `out` (level a.level - 1), no device allocation."""
        self.check(self.lib.he_ct_rescale_noalloc(self.h, a.h, out.h))
        return out

    def lincomb(self, cts, zs, target):
        """sum_i cts[i] * zs[i] at level target; zs: list of scalars or of slot vectors."""
        arr = (ctypes.c_void_p * len(cts))(*[c.h.value for c in cts])
        if np.isscalar(zs[0]):
            z = _arr(zs, np.float64)
            ns = 1
        else:
            ns = max(len(v) for v in zs)
            z = np.zeros((len(zs), ns))
            for i, v in enumerate(zs):
                z[i, :len(v)] = v
            z = _arr(z.reshape(-1), np.float64)
        return self._new(self.lib.he_ct_lincomb, arr, len(cts), _ptr(z), ns, target)

    def poly_mul(self, a, b):
        a, b = _arr(a, np.uint64), _arr(b, np.uint64)
        out = np.zeros_like(a)
        self.check(self.lib.he_poly_mul(self.h, _ptr(a), _ptr(b), a.shape[0], _ptr(out)))
        return out

    def encode(self, z, scale, nl):
        z = _arr(z, np.float64)
        out = np.zeros((nl, self.N), np.uint64)
        self.check(self.lib.he_encode(self.h, _ptr(z), len(z), scale, nl, _ptr(out)))
        return out

    # -- inference ------------------------------------------------------------
    def compile(self, layers, refresh=False, samples=1, circuit=CIRCUIT_RESTRUCTURED):
        """he_model_compile; `circuit` is he_kan_desc.circuit (CIRCUIT_PAPER runs
        the paper's order, the default applies every restructuring)."""
        return Model(self, layers, refresh, samples, circuit)

    def encrypt_input(self, model, keys, x, seed):
        """Encrypt one request's input in the model's layout: one ciphertext per
        input chunk (he_model_input_chunks), chunk c with seed + c.  For a model
        with S > 1 vectors per ciphertext x is (S, n_in) and feature i of vector
        s goes to slot i S + s."""
        b = model.input_chunks()
        S = model.samples
        x = np.asarray(x, np.float64).reshape(S, -1)
        cts = [self.encrypt(keys, x[:, lo:hi].T.reshape(-1), seed + c)
               for c, (lo, hi) in enumerate(zip(b[:-1], b[1:]))]
        return cts[0] if len(cts) == 1 else cts

    def decrypt_output(self, model, keys, ct, n_out):
        """The outputs of every vector of a request: (S, n_out) (output o of
        vector s is slot o S + s)."""
        S = model.samples
        return self.decrypt(keys, ct, n_out * S).reshape(n_out, S).T

    def eval_kan(self, model, keys, ct):
        """ct: one ciphertext, or the list of a request's input chunks."""
        if isinstance(ct, (list, tuple)):
            arr = (ctypes.c_void_p * len(ct))(*[c.h.value for c in ct])
            return self._new(self.lib.he_eval_kan_chunks, model.h, _ek(keys), arr, len(ct))
        return self._new(self.lib.he_eval_kan, model.h, _ek(keys), ct.h)

    def eval_kan_chunks(self, model, keys, cts):
        return self.eval_kan(model, keys, list(cts))

    def eval_kan_layer(self, model, keys, layer, ct):
        return self._new(self.lib.he_eval_kan_layer, model.h, _ek(keys), layer, ct.h)

    @staticmethod
    def _flat(cts):
        # requests given as ciphertexts or as lists of input chunks, request-major
        return [c for r in cts for c in (r if isinstance(r, (list, tuple)) else [r])]

    def boot(self, cts_levels, stc_levels, k_range, double_angles, cos_coeffs, real_slots=False, slots=0):
        """he_boot_create: a bootstrapping plan (see he_boot_desc; slots: a
        sparse refresh of n-periodic slot vectors, 0 for all N/2)"""
        return Boot(self, cts_levels, stc_levels, k_range, double_angles, cos_coeffs, real_slots, slots)

    def bootstrap(self, boot, keys, ct):
        return self._new(self.lib.he_bootstrap, boot.h, _ek(keys), ct.h)

    def eval_kan_boot(self, model, boot, keys, cts):
        """he_eval_kan_boot: requests (ciphertexts or lists of input chunks)
        through the network with a bootstrapping between layers"""
        n = len(cts)
        flat = self._flat(cts)
        arr = (ctypes.c_void_p * len(flat))(*[c.h.value for c in flat])
        outs = (ctypes.c_void_p * n)()
        self.check(self.lib.he_eval_kan_boot(self.h, model.h, boot.h, _ek(keys), arr, n, outs))
        return [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def boot_coeff_to_slot(self, boot, keys, ct):
        return self._new(self.lib.he_boot_coeff_to_slot, boot.h, _ek(keys), ct.h)

    def boot_eval_mod(self, boot, keys, ct):
        return self._new(self.lib.he_boot_eval_mod, boot.h, _ek(keys), ct.h)

    def boot_slot_to_coeff(self, boot, keys, ct, source_level):
        return self._new(self.lib.he_boot_slot_to_coeff, boot.h, _ek(keys), ct.h, source_level)

    def sub(self, a, b):
        return self._new(self.lib.he_ct_sub, a.h, b.h)

    def mul_i(self, a):
        return self._new(self.lib.he_ct_mul_i, a.h)

    def mod_drop(self, a, level):
        return self._new(self.lib.he_ct_mod_drop, a.h, level)

    def mod_raise(self, a):
        return self._new(self.lib.he_ct_mod_raise, a.h)

    def bootstrap_batch(self, boot, keys, cts):
        n = len(cts)
        arr = (ctypes.c_void_p * n)(*[c.h.value for c in cts])
        outs = (ctypes.c_void_p * n)()
        self.check(self.lib.he_bootstrap_batch(self.h, boot.h, _ek(keys), arr, n, outs))
        return [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def eval_kan_layer_batch(self, model, keys, layer, cts):
        n = len(cts)
        flat = self._flat(cts)
        arr = (ctypes.c_void_p * len(flat))(*[c.h.value for c in flat])
        outs = (ctypes.c_void_p * n)()
        self.check(self.lib.he_eval_kan_layer_batch(self.h, model.h, _ek(keys), layer, arr, n, outs))
        return [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def memory(self, reset_peak=False):
        v = [ctypes.c_uint64() for _ in range(3)]
        self.check(self.lib.he_ctx_memory(self.h, *[ctypes.byref(x) for x in v], 1 if reset_peak else 0))
        return {"live": v[0].value, "cached": v[1].value, "peak": v[2].value}

    def device_memory(self):
        """he_ctx_device_memory: {"free": bytes, "total": bytes} of the device."""
        f, t = ctypes.c_uint64(), ctypes.c_uint64()
        self.check(self.lib.he_ctx_device_memory(self.h, ctypes.byref(f), ctypes.byref(t)))
        return {"free": f.value, "total": t.value}

    def eval_kan_batch(self, model, keys, cts):
        n = len(cts)
        flat = self._flat(cts)
        arr = (ctypes.c_void_p * len(flat))(*[c.h.value for c in flat])
        outs = (ctypes.c_void_p * n)()
        self.check(self.lib.he_eval_kan_batch(self.h, model.h, _ek(keys), arr, n, outs))
        return [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def capture_kan_batch(self, model, keys, cts):
        """he_graph_capture_kan_batch: returns (graph, outputs); graph.launch()
        recomputes the outputs in place from the same inputs."""
        n = len(cts)
        flat = self._flat(cts)
        arr = (ctypes.c_void_p * len(flat))(*[c.h.value for c in flat])
        outs = (ctypes.c_void_p * n)()
        g = ctypes.c_void_p()
        self.check(self.lib.he_graph_capture_kan_batch(self.h, model.h, _ek(keys), arr, n, outs, ctypes.byref(g)))
        return Graph(self, g), [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]

    def graph_capture_bootstrap(self, boot, keys, cts):
        """he_graph_capture_bootstrap: (graph, outputs); each launch refreshes
        the current contents of cts into the outputs"""
        n = len(cts)
        arr = (ctypes.c_void_p * n)(*[c.h.value for c in cts])
        outs = (ctypes.c_void_p * n)()
        g = ctypes.c_void_p()
        self.check(self.lib.he_graph_capture_bootstrap(self.h, boot.h, _ek(keys), arr, n, outs, ctypes.byref(g)))
        return Graph(self, g), [Ciphertext(self, ctypes.c_void_p(outs[i])) for i in range(n)]


class NativeServer:
    """he_server_*: continuous batching by the library's own worker thread on
    the context's stream (no other thread may issue work on that context
    while the server exists)."""

    def __init__(self, ctx, keys, max_batch=16, hbm_budget=(1 << 64) - 1):
        self.ctx, self.lib = ctx, ctx.lib
        h = ctypes.c_void_p()
        ctx.check(self.lib.he_server_create(ctx.h, _ek(keys), max_batch, hbm_budget, ctypes.byref(h)))
        self.h = h

    def submit(self, model, cts):
        """One request: its ciphertext, or the list of its input chunks; returns the tag."""
        cts = list(cts) if isinstance(cts, (list, tuple)) else [cts]
        arr = (ctypes.c_void_p * len(cts))(*[c.h.value for c in cts])
        tag = ctypes.c_uint64()
        self.ctx.check(self.lib.he_submit(self.h, model.h, arr, len(cts), ctypes.byref(tag)))
        return tag.value

    def poll(self, tag, wait_ms=0):
        """(output ciphertext, ms from submission to completion), or None if
        the request has not finished within wait_ms."""
        out = ctypes.c_void_p()
        lat = ctypes.c_double()
        rc = self.lib.he_poll(self.h, tag, wait_ms, ctypes.byref(out), ctypes.byref(lat))
        if rc == HE_EAGAIN:
            return None
        if rc != HE_OK:
            raise HeError(rc, "request %d failed" % tag)
        return Ciphertext(self.ctx, out), lat.value

    def stats(self):
        v = [ctypes.c_uint64() for _ in range(3)]
        self.ctx.check(self.lib.he_server_stats(self.h, *[ctypes.byref(x) for x in v]))
        return {"completed": v[0].value, "layer_batches": v[1].value, "layer_runs": v[2].value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.he_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Graph:
    """A captured batched inference (he_graph_*)."""

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def launch(self):
        self.ctx.check(self.ctx.lib.he_graph_launch(self.h))

    def free(self):
        if self.h:
            self.ctx.check(self.ctx.lib.he_graph_free(self.h))
            self.h = None


class SecretKey:
    """he_secret_key (client side, host memory)."""

    def __init__(self, ctx, h):
        self.ctx, self.h, self.lib = ctx, h, ctx.lib

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.he_secret_key_free(self.h)
            self.h = None


class EvalKeys:
    """he_eval_keys (server side: relinearisation and Galois keys, no secret)."""

    def __init__(self, ctx, h):
        self.ctx, self.h, self.lib = ctx, h, ctx.lib

    def ids(self):
        n = ctypes.c_size_t()
        self.ctx.check(self.lib.he_eval_keys_ids(self.h, None, 0, ctypes.byref(n)))
        v = (ctypes.c_uint32 * max(1, n.value))()
        self.ctx.check(self.lib.he_eval_keys_ids(self.h, v, n.value, ctypes.byref(n)))
        return [int(v[i]) for i in range(n.value)]

    def export(self, key_id, digit):
        c = self.ctx
        ktot = c.L + 1 + c.alpha
        out = np.zeros((2, ktot, c.N), np.uint64)
        c.check(self.lib.he_eval_keys_export(c.h, self.h, key_id, digit, _ptr(out), out.size))
        return out

    def export_all(self):
        """{key id: [dnum][2][L+1+alpha][N] residues}: what a client sends a server."""
        c = self.ctx
        dnum = (c.L + 1 + c.w - 1) // c.w
        return {i: np.stack([self.export(i, j) for j in range(dnum)]) for i in self.ids()}

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.he_eval_keys_free(self.h)
            self.h = None


class Keys:
    """A client's key pair from keygen: .sk and .ek; export() reads the
    evaluation keys."""

    def __init__(self, sk, ek):
        self.sk, self.ek = sk, ek
        self.ctx = ek.ctx

    def export(self, key_id, digit):
        return self.ek.export(key_id, digit)


def _sk(keys):
    k = keys.sk if isinstance(keys, Keys) else keys
    if not isinstance(k, SecretKey):
        raise TypeError("a secret key is needed")
    return k.h


def _ek(keys):
    k = keys.ek if isinstance(keys, Keys) else keys
    if not isinstance(k, EvalKeys):
        raise TypeError("evaluation keys are needed")
    return k.h


class Ciphertext:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    @property
    def level(self):
        return self.ctx.lib.he_ct_level(self.h)

    def export(self):
        c = self.ctx
        l = self.level
        out = np.zeros((2, l + 1, c.N), np.uint64)
        c.check(c.lib.he_ct_export(c.h, self.h, _ptr(out), out.size))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.he_ct_free(self.h)
            self.h = None


class Boot:
    """A bootstrapping plan (he_boot_create)."""

    def __init__(self, ctx, cts_levels, stc_levels, k_range, double_angles, cos_coeffs, real_slots=False, slots=0):
        self.ctx = ctx
        cf = _arr(cos_coeffs, np.float64)
        desc = he_boot_desc(cts_levels, stc_levels, float(k_range), double_angles, len(cf) - 1, _ptr(cf),
                            1 if real_slots else 0, int(slots))
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.he_boot_create(ctx.h, ctypes.byref(desc), ctypes.byref(h)))
        self.h = h

    def rotation_steps(self):
        n = ctypes.c_size_t()
        self.ctx.check(self.ctx.lib.he_boot_rotation_steps(self.h, None, 0, ctypes.byref(n)))
        s = np.zeros(n.value, np.int32)
        self.ctx.check(self.ctx.lib.he_boot_rotation_steps(self.h, _ptr(s), n.value, ctypes.byref(n)))
        return [int(v) for v in s]

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.he_boot_free(self.h)
            self.h = None


class Model:
    def __init__(self, ctx, layers, refresh=False, samples=1, circuit=CIRCUIT_RESTRUCTURED):
        self.ctx = ctx
        self.samples = samples
        self.circuit = circuit
        keep = []
        arr = (he_kan_layer * len(layers))()
        for i, L in enumerate(layers):
            f = lambda a: keep.append(_arr(a, np.float64)) or keep[-1]
            knots, wb, ws, c = f(L.knots), f(L.wb), f(L.ws), f(L.c)
            sc = f(L.silu_coeffs)
            lens = _arr([len(s) for s in L.comp], np.int32)
            keep.append(lens)
            cc = f(np.concatenate([np.asarray(s, np.float64) for s in L.comp]))
            arr[i] = he_kan_layer(L.n_in, L.n_out, L.g, L.k, _ptr(knots), _ptr(wb), _ptr(ws), _ptr(c),
                                  len(sc) - 1, _ptr(sc), L.silu_lo, L.silu_hi, len(L.comp), _ptr(lens), _ptr(cc),
                                  float(getattr(L, "comp_prescale", 0.0)))
        desc = he_kan_desc(len(layers), arr, samples, circuit)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.he_model_compile(ctx.h, ctypes.byref(desc), 1 if refresh else 0, ctypes.byref(h)))
        self.h = h
        self.n_layers = len(layers)

    def input_chunks(self):
        """Feature bounds [b_0 = 0, b_1, ..., b_nc = n_in] of the input chunks."""
        n = ctypes.c_size_t()
        self.ctx.check(self.ctx.lib.he_model_input_chunks(self.h, None, 0, ctypes.byref(n)))
        b = np.zeros(n.value + 1, np.int32)
        self.ctx.check(self.ctx.lib.he_model_input_chunks(self.h, _ptr(b), n.value + 1, ctypes.byref(n)))
        return [int(v) for v in b]

    def output_period(self, layer):
        """he_model_output_period: the period of the layer's output slots"""
        v = ctypes.c_int64()
        self.ctx.check(self.ctx.lib.he_model_output_period(self.h, layer, ctypes.byref(v)))
        return v.value

    def rotation_steps(self):
        n = ctypes.c_size_t()
        self.ctx.check(self.ctx.lib.he_model_rotation_steps(self.h, None, 0, ctypes.byref(n)))
        s = np.zeros(n.value, np.int32)
        self.ctx.check(self.ctx.lib.he_model_rotation_steps(self.h, _ptr(s), n.value, ctypes.byref(n)))
        return [int(v) for v in s]

    def __del__(self):
        if getattr(self, "h", None):
            self.ctx.lib.he_model_free(self.h)
            self.h = None
