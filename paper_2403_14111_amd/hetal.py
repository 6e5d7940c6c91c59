"""Python binding of libhetal.so (include/hetal.h): argument marshalling only.

Device memory for ciphertexts, plaintexts and matrices comes from PyTorch
(torch tensors on the current CUDA/HIP device, holding the 64-bit words); the
library's HIP stream is PyTorch's current stream at context creation.  Every
computation runs in the library's kernels.  If the library is not built, the
import fails loudly: there is no other implementation behind these calls.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libhetal.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhetal.so is not built (%s); run __graft_entry__.build() or "
                      "python paper_2403_14111_amd/build.py" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
ERRORS = {-1: "E_INVALID_ARG", -2: "E_SHAPE", -3: "E_LEVEL", -4: "E_NO_KEY", -5: "E_SCALE", -6: "E_OOM",
          -7: "E_DEVICE", -8: "E_PARAMS", -9: "E_OVERFLOW"}


class HetalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int), ("num_q", ctypes.c_int), ("num_p", ctypes.c_int), ("dnum", ctypes.c_int),
                ("q0_bits", ctypes.c_int), ("q_bits", ctypes.c_int)]


class _Ct(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("capacity", ctypes.c_size_t), ("level", ctypes.c_int),
                ("scale", ctypes.c_double)]


class _Mat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("capacity", ctypes.c_size_t), ("n_rb", ctypes.c_int),
                ("n_cb", ctypes.c_int), ("s0", ctypes.c_int), ("s1", ctypes.c_int), ("level", ctypes.c_int),
                ("scale", ctypes.c_double)]


class _Tune(ctypes.Structure):
    _fields_ = [("ks_group", ctypes.c_int), ("tpt_modup", ctypes.c_int), ("tpt_moddown", ctypes.c_int),
                ("two_streams", ctypes.c_int), ("work_cts", ctypes.c_int)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("untuned_ms", ctypes.c_double), ("tuned_ms", ctypes.c_double), ("classes", ctypes.c_int),
                ("trials", ctypes.c_int), ("two_streams", ctypes.c_int)]


class _Req(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("a", ctypes.POINTER(_Mat)), ("b", ctypes.POINTER(_Mat)), ("c", ctypes.c_int),
                ("t", ctypes.c_double)]


class SoftmaxParams(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("L", ctypes.c_double), ("n", ctypes.c_int), ("precise", ctypes.c_int),
                ("extend", ctypes.c_int), ("comp_g", ctypes.c_int), ("exp_B", ctypes.c_int),
                ("exp_degree", ctypes.c_int), ("exp_coeffs", ctypes.c_double * 32), ("inv_R", ctypes.c_double),
                ("inv_iters", ctypes.c_int)]


REFRESH_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(_Ct))

_vp = ctypes.c_void_p
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dblp = ctypes.POINTER(ctypes.c_double)
_intp = ctypes.POINTER(ctypes.c_int)
_ctp = ctypes.POINTER(_Ct)
_matp = ctypes.POINTER(_Mat)

_SIGS = {
    "hetal_last_error": (ctypes.c_char_p, []),
    "hetal_ctx_create": (ctypes.c_int, [ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "hetal_ctx_destroy": (None, [_vp]),
    "hetal_ctx_set_stream": (ctypes.c_int, [_vp, _vp]),
    "hetal_ctx_info": (ctypes.c_int, [_vp, _intp, _intp, _intp, _intp]),
    "hetal_ctx_primes": (ctypes.c_int, [_vp, _u64p]),
    "hetal_synchronize": (ctypes.c_int, [_vp]),
    "hetal_galois_rot": (ctypes.c_uint64, [_vp, ctypes.c_int]),
    "hetal_galois_conj": (ctypes.c_uint64, [_vp]),
    "hetal_sk_create": (ctypes.c_int, [_vp, _i64p, ctypes.POINTER(_vp)]),
    "hetal_sk_destroy": (None, [_vp]),
    "hetal_keys_create": (ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    "hetal_keys_destroy": (None, [_vp]),
    "hetal_keys_gen_relin": (ctypes.c_int, [_vp, _vp, _vp, _u64p, _i64p]),
    "hetal_keys_gen_galois": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_uint64, _u64p, _i64p]),
    "hetal_encode": (ctypes.c_int, [_vp, _dblp, _dblp, ctypes.c_int, ctypes.c_double, _ctp]),
    "hetal_decode": (ctypes.c_int, [_vp, _ctp, _dblp, _dblp]),
    "hetal_encrypt": (ctypes.c_int, [_vp, _vp, _ctp, _u64p, _i64p, _ctp]),
    "hetal_encrypt_seeded": (ctypes.c_int, [_vp, _vp, _ctp, ctypes.c_uint64, ctypes.c_uint32, _ctp]),
    "hetal_keygen": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "hetal_ctx_create_shared": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    "hetal_ctx_set_two_streams": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hetal_gen_evk": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int]),
    "hetal_gaussian_table": (ctypes.c_int, [_u64p, ctypes.POINTER(ctypes.c_int)]),
    "hetal_sample_ternary": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, _i64p]),
    "hetal_sample_uniform": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                            ctypes.c_int, _u64p]),
    "hetal_sample_gaussian": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                             _i64p]),
    "hetal_decrypt": (ctypes.c_int, [_vp, _vp, _ctp, _ctp]),
    "hetal_add": (ctypes.c_int, [_vp, _ctp, _ctp, _ctp]),
    "hetal_sub": (ctypes.c_int, [_vp, _ctp, _ctp, _ctp]),
    "hetal_mul_i": (ctypes.c_int, [_vp, _ctp, _ctp]),
    "hetal_cmult": (ctypes.c_int, [_vp, _ctp, _ctp, _ctp]),
    "hetal_hmult": (ctypes.c_int, [_vp, _vp, _ctp, _ctp, _ctp]),
    "hetal_hrot": (ctypes.c_int, [_vp, _vp, _ctp, ctypes.c_int, _ctp]),
    "hetal_hrot_batch": (ctypes.c_int, [_vp, _vp, _ctp, _intp, ctypes.c_int, _ctp]),
    "hetal_hrot_noalloc": (ctypes.c_int, [_vp, _vp, _ctp, ctypes.c_int, _ctp]),
    "hetal_conj": (ctypes.c_int, [_vp, _vp, _ctp, _ctp]),
    "hetal_rescale": (ctypes.c_int, [_vp, _ctp, _ctp]),
    "hetal_mod_drop": (ctypes.c_int, [_vp, _ctp, ctypes.c_int, _ctp]),
    "hetal_ct_to_coeff": (ctypes.c_int, [_vp, _ctp, _u64p]),
    "hetal_pt_to_coeff": (ctypes.c_int, [_vp, _ctp, _u64p]),
    "hetal_ct_from_coeff": (ctypes.c_int, [_vp, _u64p, ctypes.c_int, ctypes.c_double, _ctp]),
    "hetal_mat_encrypt": (ctypes.c_int, [_vp, _vp, _dblp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _u64p, _i64p, _matp]),
    "hetal_mat_encrypt_seeded": (ctypes.c_int, [_vp, _vp, _dblp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _matp]),
    "hetal_mat_decrypt": (ctypes.c_int, [_vp, _vp, _matp, _dblp]),
    "hetal_enc_matmul_abt": (ctypes.c_int, [_vp, _vp, _matp, _matp, ctypes.c_int, ctypes.c_double, _matp]),
    "hetal_enc_matmul_atb": (ctypes.c_int, [_vp, _vp, _matp, _matp, ctypes.c_int, ctypes.c_double, _matp]),
    "hetal_enc_matmul_batch": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_Req), ctypes.c_int, _matp]),
    "hetal_autotune_batch": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_Req), ctypes.c_int, _matp, ctypes.c_int,
                                            ctypes.POINTER(_TuneReport)]),
    "hetal_tune_get": (ctypes.c_int, [_vp] + [ctypes.c_int] * 5 + [ctypes.POINTER(_Tune)]),
    "hetal_tune_set": (ctypes.c_int, [_vp] + [ctypes.c_int] * 5 + [ctypes.POINTER(_Tune)]),
    "hetal_tune_reset": (ctypes.c_int, [_vp]),
    "hetal_required_rot_steps": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _intp]),
    "hetal_enc_matmul_batch_graph": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_Req), ctypes.c_int, _matp,
                                                    ctypes.POINTER(_vp)]),
    "hetal_graph_launch": (ctypes.c_int, [_vp]),
    "hetal_graph_destroy": (None, [_vp]),
    "hetal_cmult_const": (ctypes.c_int, [_vp, _ctp, ctypes.c_double, ctypes.c_double, _ctp]),
    "hetal_add_const": (ctypes.c_int, [_vp, _ctp, ctypes.c_double, _ctp]),
    "hetal_add_plain": (ctypes.c_int, [_vp, _ctp, _ctp, _ctp]),
    "hetal_refresh": (ctypes.c_int, [_vp, _vp, _ctp, ctypes.c_double, _u64p, _i64p, _ctp]),
    "hetal_poly_eval": (ctypes.c_int, [_vp, _vp, _ctp, _dblp, ctypes.c_int, REFRESH_FN, _vp, _ctp]),
    "hetal_softmax_default_params": (ctypes.c_int, [ctypes.POINTER(SoftmaxParams)]),
    "hetal_softmax_rot_steps": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _i32p, _intp]),
    "hetal_softmax_approx": (ctypes.c_int, [_vp, _vp, _matp, ctypes.c_int, ctypes.POINTER(SoftmaxParams), REFRESH_FN,
                                            _vp, _matp, _intp]),
    "hetal_nag_step": (ctypes.c_int, [_vp, _vp, _matp, _matp, _matp, _matp, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(SoftmaxParams), REFRESH_FN, _vp, _matp, _matp,
                                      _intp]),
    "hetal_counters_get": (ctypes.c_int, [_vp, _i64p]),
    "hetal_counters_reset": (ctypes.c_int, [_vp]),
    "hetal_ks_counts": (ctypes.c_int, [_vp, _i64p, _i64p, ctypes.c_int]),
    "hetal_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "hetal_timing_classes": (ctypes.c_int, []),
    "hetal_timing_get": (ctypes.c_int, [_vp, _dblp, _i64p, _dblp]),
}

KERNEL_CLASSES = ["ntt_fwd_strided", "ks_modup", "ks_moddown", "ntt_fwd_contig", "ntt_fwd_epilogue",
                  "ntt_inv_contig", "ntt_inv_strided", "ks_inner", "rescale", "elementwise", "encode"]
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return sorted(_SIGS)


def _check(rc):
    if rc != OK:
        raise HetalError(rc, _lib.hetal_last_error().decode())


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_u64p)


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _dbl(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dblp)


PRESETS = {
    # 2^12 ring, q_0 (50-bit) + 4 x 40-bit, one special prime, one prime per digit.
    "toy": dict(log_n=12, num_q=5, num_p=1, dnum=5, q0_bits=50, q_bits=40),
    # 2^16 ring, q_0 (50-bit) + 11 x 40-bit, three special primes, dnum = 4.
    "n16l12": dict(log_n=16, num_q=12, num_p=3, dnum=4, q0_bits=50, q_bits=40),
    # 2^12 ring with the 2^16 ring's modulus chain shape (deep pipelines at test sizes).
    "n12l12": dict(log_n=12, num_q=12, num_p=3, dnum=4, q0_bits=50, q_bits=40),
}


def softmax_default_params():
    p = SoftmaxParams()
    _check(_lib.hetal_softmax_default_params(ctypes.byref(p)))
    return p


class Ciphertext:
    """Device buffer ([2][level+1][N] words) + level + scale.  Also used for plaintexts ([level+1][N]).
    `buf` may be a view into a larger tensor (see Context.new_ct_batch)."""

    def __init__(self, ctx, level, words, scale=0.0, buf=None):
        self.ctx = ctx
        self.buf = torch.empty(words, dtype=torch.int64, device=ctx.device) if buf is None else buf
        self.level = level
        self.scale = scale

    def _struct(self):
        return _Ct(self.buf.data_ptr(), self.buf.numel(), self.level, self.scale)


class Matrix:
    def __init__(self, ctx, words, s0, level, scale):
        self.ctx = ctx
        self.buf = torch.empty(max(words, 1), dtype=torch.int64, device=ctx.device)
        self.n_rb = self.n_cb = 0
        self.s0 = s0
        self.s1 = ctx.slots // s0
        self.level = level
        self.scale = scale

    def _struct(self):
        return _Mat(self.buf.data_ptr(), self.buf.numel(), self.n_rb, self.n_cb, self.s0, self.s1, self.level,
                    self.scale)

    def _update(self, m):
        self.n_rb, self.n_cb, self.s0, self.s1, self.level, self.scale = m.n_rb, m.n_cb, m.s0, m.s1, m.level, m.scale


def gaussian_table():
    """The error sampler's 19 cumulative thresholds (hetal_gaussian_table)."""
    out = np.empty(19, dtype=np.uint64)
    n = ctypes.c_int(19)
    _check(_lib.hetal_gaussian_table(out.ctypes.data_as(_u64p), ctypes.byref(n)))
    return out[:n.value]


def sample_ternary(log_n, seed, h):
    out = np.empty(1 << log_n, dtype=np.int64)
    _check(_lib.hetal_sample_ternary(int(log_n), int(seed), int(h), out.ctypes.data_as(_i64p)))
    return out


class Context:
    def __init__(self, preset="toy", device="cuda:0", **overrides):
        if not torch.cuda.is_available():
            raise RuntimeError("the HETAL library needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        cfg = dict(PRESETS[preset]) if isinstance(preset, str) else dict(preset)
        cfg.update(overrides)
        self.params = Params(**cfg)
        self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        _check(_lib.hetal_ctx_create(ctypes.byref(self.params), _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        n, slots, ml, npr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.hetal_ctx_info(h, ctypes.byref(n), ctypes.byref(slots), ctypes.byref(ml), ctypes.byref(npr)))
        self.n, self.slots, self.max_level, self.num_primes = n.value, slots.value, ml.value, npr.value
        pr = np.zeros(self.num_primes, dtype=np.uint64)
        _check(_lib.hetal_ctx_primes(h, pr.ctypes.data_as(_u64p)))
        self.primes = [int(x) for x in pr]
        self.num_q = cfg["num_q"]
        self.num_p = cfg["num_p"]
        self.dnum = cfg["dnum"]
        self.q = self.primes[:self.num_q]
        self.p = self.primes[self.num_q:]

    def share(self, stream):
        """A context on the torch stream `stream` sharing this one's parameters, tables and keys
        (hetal_ctx_create_shared); this context must outlive it."""
        other = object.__new__(Context)
        other.__dict__.update({k: v for k, v in self.__dict__.items() if k != "_h"})
        other.stream = stream
        other.base = self
        h = _vp()
        _check(_lib.hetal_ctx_create_shared(self._h, _vp(stream.cuda_stream), ctypes.byref(h)))
        other._h = h
        return other

    def set_two_streams(self, on):
        """Whether batched products may use the context's second stream (hetal_ctx_set_two_streams)."""
        _check(_lib.hetal_ctx_set_two_streams(self._h, int(bool(on))))

    # The destroy functions are bound as default arguments: at interpreter shutdown the module's globals
    # (_lib included) may already be cleared when the last handles are collected.
    def __del__(self, _destroy=_lib.hetal_ctx_destroy):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)

    # -- sizes / buffers --
    def ct_words(self, level):
        return 2 * (level + 1) * self.n

    def new_ct(self, level):
        return Ciphertext(self, level, self.ct_words(level))

    def new_ct_batch(self, count, level):
        """`count` ciphertexts at `level` laid out back to back in one device buffer."""
        w = self.ct_words(level)
        big = torch.empty(max(count, 1) * w, dtype=torch.int64, device=self.device)
        return [Ciphertext(self, level, w, buf=big[i * w:(i + 1) * w]) for i in range(count)]

    def new_pt(self, level):
        return Ciphertext(self, level, (level + 1) * self.n)

    def galois_rot(self, r):
        return int(_lib.hetal_galois_rot(self._h, int(r)))

    def galois_conj(self):
        return int(_lib.hetal_galois_conj(self._h))

    def synchronize(self):
        _check(_lib.hetal_synchronize(self._h))

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        _check(_lib.hetal_counters_get(self._h, out.ctypes.data_as(_i64p)))
        return dict(zip(["rot", "conj", "mult", "cmult", "rescale", "keyswitch", "ntt_limbs", "launches"],
                        [int(x) for x in out]))

    def ks_counts(self):
        """Key switches by input level since the last reset: (items, key_reads), each a list per level."""
        items = np.zeros(self.max_level + 1, dtype=np.int64)
        reads = np.zeros(self.max_level + 1, dtype=np.int64)
        _check(_lib.hetal_ks_counts(self._h, items.ctypes.data_as(_i64p), reads.ctypes.data_as(_i64p),
                                    self.max_level + 1))
        return [int(v) for v in items], [int(v) for v in reads]

    def reset_counters(self):
        _check(_lib.hetal_counters_reset(self._h))

    def timing_enable(self, on=True):
        _check(_lib.hetal_timing_enable(self._h, 1 if on else 0))

    def timing_get(self):
        k = _lib.hetal_timing_classes()
        if k != len(KERNEL_CLASSES):
            raise HetalError(-1, "library reports %d timing classes, binding knows %d" % (k, len(KERNEL_CLASSES)))
        ms = np.zeros(k)
        n = np.zeros(k, dtype=np.int64)
        b = np.zeros(k)
        _check(_lib.hetal_timing_get(self._h, ms.ctypes.data_as(_dblp), n.ctypes.data_as(_i64p),
                                     b.ctypes.data_as(_dblp)))
        return {k: dict(ms=float(ms[i]), launches=int(n[i]), bytes=float(b[i])) for i, k in enumerate(KERNEL_CLASSES)}

    # -- keys --
    def sk_create(self, s_coeffs):
        s, sp = _i64(s_coeffs)
        assert s.shape == (self.n,)
        return SecretKey(self, s, sp)

    def keys_create(self):
        return KeySet(self)

    def keygen(self, seed):
        """The secret key drawn by the library from `seed` (hetal_keygen)."""
        return SecretKey(self, None, None, seed=seed)

    # -- the library's seeded sampler (for tests and callers that keep their own randomness) --
    def sample_uniform(self, seed, purpose, index, rows, group):
        out = np.empty((rows, self.n), dtype=np.uint64)
        _check(_lib.hetal_sample_uniform(self._h, int(seed), int(purpose), int(index), int(rows), int(group),
                                         out.ctypes.data_as(_u64p)))
        return out

    def sample_gaussian(self, seed, purpose, index, count):
        out = np.empty((count, self.n), dtype=np.int64)
        _check(_lib.hetal_sample_gaussian(self._h, int(seed), int(purpose), int(index), int(count),
                                          out.ctypes.data_as(_i64p)))
        return out

    # -- encoding / encryption --
    def encode(self, z, level, scale):
        z = np.asarray(z, dtype=np.complex128)
        assert z.shape == (self.slots,)
        re, rp = _dbl(z.real)
        im, ip = _dbl(z.imag)
        pt = self.new_pt(level)
        s = pt._struct()
        _check(_lib.hetal_encode(self._h, rp, ip, level, float(scale), ctypes.byref(s)))
        pt.level, pt.scale = s.level, s.scale
        return pt

    def decode(self, pt):
        re = np.empty(self.slots)
        im = np.empty(self.slots)
        s = pt._struct()
        _check(_lib.hetal_decode(self._h, ctypes.byref(s), re.ctypes.data_as(_dblp), im.ctypes.data_as(_dblp)))
        return re + 1j * im

    def encrypt(self, sk, pt, a, e):
        a, ap = _u64(a)
        e, ep = _i64(e)
        assert a.shape == (pt.level + 1, self.n) and e.shape == (self.n,)
        out = self.new_ct(pt.level)
        s = out._struct()
        _check(_lib.hetal_encrypt(self._h, sk._h, ctypes.byref(pt._struct()), ap, ep, ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def encrypt_seeded(self, sk, pt, seed, index):
        out = self.new_ct(pt.level)
        s = out._struct()
        _check(_lib.hetal_encrypt_seeded(self._h, sk._h, ctypes.byref(pt._struct()), int(seed), int(index),
                                         ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def decrypt(self, sk, ct):
        pt = self.new_pt(ct.level)
        s = pt._struct()
        _check(_lib.hetal_decrypt(self._h, sk._h, ctypes.byref(ct._struct()), ctypes.byref(s)))
        pt.level, pt.scale = s.level, s.scale
        return pt

    # -- homomorphic operations --
    def _unary(self, fn, a, out_level, *args):
        out = self.new_ct(out_level)
        s = out._struct()
        _check(fn(self._h, *args, ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def add(self, a, b):
        return self._unary(_lib.hetal_add, a, a.level, ctypes.byref(a._struct()), ctypes.byref(b._struct()))

    def sub(self, a, b):
        return self._unary(_lib.hetal_sub, a, a.level, ctypes.byref(a._struct()), ctypes.byref(b._struct()))

    def mul_i(self, a):
        return self._unary(_lib.hetal_mul_i, a, a.level, ctypes.byref(a._struct()))

    def cmult(self, a, pt):
        return self._unary(_lib.hetal_cmult, a, a.level, ctypes.byref(a._struct()), ctypes.byref(pt._struct()))

    def hmult(self, keys, a, b):
        out = self.new_ct(a.level)
        s = out._struct()
        _check(_lib.hetal_hmult(self._h, keys._h, ctypes.byref(a._struct()), ctypes.byref(b._struct()),
                                ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def hrot(self, keys, a, r):
        out = self.new_ct(a.level)
        s = out._struct()
        _check(_lib.hetal_hrot(self._h, keys._h, ctypes.byref(a._struct()), int(r), ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def hrot_noalloc(self, keys, a, r, out):
        """hrot into the caller's `out` (not `a`) with the key switch's temporaries in the library's fixed
        device scratch region: the call allocates no device memory."""
        s = out._struct()
        _check(_lib.hetal_hrot_noalloc(self._h, keys._h, ctypes.byref(a._struct()), int(r), ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def hrot_batch(self, keys, cts, steps, out=None):
        """[Lrot(cts[i], steps[i])] as one batched key switch (steps: one int for all, or one per item)."""
        n = len(cts)
        steps = [int(steps)] * n if np.ndim(steps) == 0 else [int(s) for s in steps]
        if len(steps) != n:
            raise ValueError("one step per ciphertext")
        if n == 0:
            return []
        out = self.new_ct_batch(n, cts[0].level) if out is None else out
        ins = (_Ct * n)(*[c._struct() for c in cts])
        outs = (_Ct * n)(*[o._struct() for o in out])
        st = (ctypes.c_int * n)(*steps)
        _check(_lib.hetal_hrot_batch(self._h, keys._h, ins, st, n, outs))
        for o, s in zip(out, outs):
            o.level, o.scale = s.level, s.scale
        return out

    def conj(self, keys, a):
        out = self.new_ct(a.level)
        s = out._struct()
        _check(_lib.hetal_conj(self._h, keys._h, ctypes.byref(a._struct()), ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def rescale(self, a):
        return self._unary(_lib.hetal_rescale, a, max(a.level - 1, 0), ctypes.byref(a._struct()))

    def mod_drop(self, a, level):
        return self._unary(_lib.hetal_mod_drop, a, max(min(level, a.level), 0), ctypes.byref(a._struct()),
                           int(level))

    # -- canonical forms --
    def ct_to_coeff(self, ct):
        out = np.empty((2, ct.level + 1, self.n), dtype=np.uint64)
        _check(_lib.hetal_ct_to_coeff(self._h, ctypes.byref(ct._struct()), out.ctypes.data_as(_u64p)))
        return out

    def pt_to_coeff(self, pt):
        out = np.empty((pt.level + 1, self.n), dtype=np.uint64)
        _check(_lib.hetal_pt_to_coeff(self._h, ctypes.byref(pt._struct()), out.ctypes.data_as(_u64p)))
        return out

    def ct_from_coeff(self, coeffs, scale):
        c, cp = _u64(coeffs)
        level = c.shape[1] - 1
        out = self.new_ct(level)
        s = out._struct()
        _check(_lib.hetal_ct_from_coeff(self._h, cp, level, float(scale), ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    # -- matrices --
    def mat_blocks(self, rows, cols, s0, tiling=0, c=1):
        s1 = self.slots // s0
        if tiling == 1:
            return 1, -(-cols // s1)
        if tiling == 2:
            return -(-rows // s0), 1
        return -(-rows // s0), -(-cols // s1)

    def mat_encrypt(self, sk, mat, s0, level, scale, a, e, tiling=0, c=1):
        mat, mp = _dbl(mat)
        rows, cols = mat.shape
        n_rb, n_cb = self.mat_blocks(rows, cols, s0, tiling, c)
        a, ap = _u64(a)
        e, ep = _i64(e)
        assert a.shape == (n_rb * n_cb, level + 1, self.n) and e.shape == (n_rb * n_cb, self.n), (a.shape, e.shape)
        m = Matrix(self, n_rb * n_cb * self.ct_words(level), s0, level, scale)
        s = m._struct()
        _check(_lib.hetal_mat_encrypt(self._h, sk._h, mp, rows, cols, int(tiling), int(c), ap, ep, ctypes.byref(s)))
        m._update(s)
        return m

    def mat_encrypt_seeded(self, sk, mat, s0, level, scale, seed, first_index, tiling=0, c=1):
        mat, mp = _dbl(mat)
        rows, cols = mat.shape
        n_rb, n_cb = self.mat_blocks(rows, cols, s0, tiling, c)
        m = Matrix(self, n_rb * n_cb * self.ct_words(level), s0, level, scale)
        s = m._struct()
        _check(_lib.hetal_mat_encrypt_seeded(self._h, sk._h, mp, rows, cols, int(tiling), int(c), int(seed),
                                             int(first_index), ctypes.byref(s)))
        m._update(s)
        return m

    def mat_decrypt(self, sk, m):
        out = np.empty((m.n_rb * m.s0, m.n_cb * m.s1))
        _check(_lib.hetal_mat_decrypt(self._h, sk._h, ctypes.byref(m._struct()), out.ctypes.data_as(_dblp)))
        return out

    def mat_block(self, m, b):
        """Ciphertext view of block b (shares the matrix's memory)."""
        w = self.ct_words(m.level)
        ct = Ciphertext.__new__(Ciphertext)
        ct.ctx, ct.buf, ct.level, ct.scale = self, m.buf[b * w:(b + 1) * w], m.level, m.scale
        return ct

    def enc_matmul_abt(self, keys, a, bbar, c, t=1.0):
        out = Matrix(self, a.n_rb * self.ct_words(min(a.level, bbar.level) - 3) if min(a.level, bbar.level) >= 3
                     else 1, a.s0, 0, 0.0)
        s = out._struct()
        _check(_lib.hetal_enc_matmul_abt(self._h, keys._h, ctypes.byref(a._struct()), ctypes.byref(bbar._struct()),
                                         int(c), float(t), ctypes.byref(s)))
        out._update(s)
        return out

    def enc_matmul_batch(self, keys, reqs, _autotune_reps=0):
        """[(op, a, b, c, t), ...] with op "abt" or "atb" -> the list of results, each exactly what
        enc_matmul_abt / enc_matmul_atb returns for it; requests sharing (op, c, s0, levels, scales) run in lockstep."""
        n = len(reqs)
        mats, outs = [], []
        arr = (_Req * max(n, 1))()
        for i, (op, a, b, c, t) in enumerate(reqs):
            if op not in ("abt", "atb"):
                raise ValueError("op must be 'abt' or 'atb'")
            sa, sb = a._struct(), b._struct()
            mats += [sa, sb]
            if op == "abt":
                lv = min(a.level, b.level) - 3
                out = Matrix(self, a.n_rb * self.ct_words(lv) if lv >= 0 else 1, a.s0, 0, 0.0)
            else:
                out = Matrix(self, b.n_cb * self.ct_words(max(a.level, b.level)), b.s0, 0, 0.0)
            outs.append(out)
            arr[i] = _Req(0 if op == "abt" else 1, ctypes.pointer(sa), ctypes.pointer(sb), int(c), float(t))
        structs = (_Mat * max(n, 1))(*[o._struct() for o in outs])
        if _autotune_reps:
            rep = _TuneReport()
            _check(_lib.hetal_autotune_batch(self._h, keys._h, arr, n, structs, int(_autotune_reps),
                                             ctypes.byref(rep)))
            self.last_tune_report = dict(untuned_ms=rep.untuned_ms, tuned_ms=rep.tuned_ms, classes=rep.classes,
                                         trials=rep.trials, two_streams=bool(rep.two_streams))
        else:
            _check(_lib.hetal_enc_matmul_batch(self._h, keys._h, arr, n, structs))
        for o, s in zip(outs, structs):
            o._update(s)
        return outs

    def autotune_batch(self, keys, reqs, reps=3):
        """The autotuner (hetal_autotune_batch) on this batch: -> (outputs, report); later batches of these shape
        classes run with the chosen schedules."""
        outs = self.enc_matmul_batch(keys, reqs, _autotune_reps=reps)
        return outs, self.last_tune_report

    def tune_get(self, op, c, s0, level_a, level_b):
        t = _Tune()
        _check(_lib.hetal_tune_get(self._h, 0 if op == "abt" else 1, int(c), int(s0), int(level_a), int(level_b),
                                   ctypes.byref(t)))
        return dict(ks_group=t.ks_group, tpt_modup=t.tpt_modup, tpt_moddown=t.tpt_moddown,
                    two_streams=bool(t.two_streams), work_cts=t.work_cts)

    def tune_set(self, op, c, s0, level_a, level_b, ks_group=32, tpt_modup=0, tpt_moddown=0, two_streams=True,
                 work_cts=0):
        t = _Tune(int(ks_group), int(tpt_modup), int(tpt_moddown), int(bool(two_streams)), int(work_cts))
        _check(_lib.hetal_tune_set(self._h, 0 if op == "abt" else 1, int(c), int(s0), int(level_a), int(level_b),
                                   ctypes.byref(t)))

    def tune_reset(self):
        _check(_lib.hetal_tune_reset(self._h))

    def enc_matmul_batch_graph(self, keys, reqs):
        """enc_matmul_batch recorded into a HIP graph -> (outputs, graph); graph.launch() recomputes the outputs
        from the inputs' current contents.  The inputs, outputs and keys must stay alive while the graph is."""
        n = len(reqs)
        outs, keep = [], []
        arr = (_Req * max(n, 1))()
        for i, (op, a, b, c, t) in enumerate(reqs):
            if op not in ("abt", "atb"):
                raise ValueError("op must be 'abt' or 'atb'")
            sa, sb = a._struct(), b._struct()
            keep += [sa, sb, a, b]
            if op == "abt":
                lv = min(a.level, b.level) - 3
                out = Matrix(self, a.n_rb * self.ct_words(lv) if lv >= 0 else 1, a.s0, 0, 0.0)
            else:
                out = Matrix(self, b.n_cb * self.ct_words(max(a.level, b.level)), b.s0, 0, 0.0)
            outs.append(out)
            arr[i] = _Req(0 if op == "abt" else 1, ctypes.pointer(sa), ctypes.pointer(sb), int(c), float(t))
        structs = (_Mat * max(n, 1))(*[o._struct() for o in outs])
        h = _vp()
        _check(_lib.hetal_enc_matmul_batch_graph(self._h, keys._h, arr, n, structs, ctypes.byref(h)))
        for o, s in zip(outs, structs):
            o._update(s)
        return outs, Graph(self, h, keep + outs + [keys])

    def enc_matmul_atb(self, keys, abar, b, c, t=1.0):
        lvl = max(abar.level, b.level)
        out = Matrix(self, b.n_cb * self.ct_words(lvl), b.s0, 0, 0.0)
        s = out._struct()
        _check(_lib.hetal_enc_matmul_atb(self._h, keys._h, ctypes.byref(abar._struct()), ctypes.byref(b._struct()),
                                         int(c), float(t), ctypes.byref(s)))
        out._update(s)
        return out

    # -- constants, refresh, polynomials, softmax (App. softmax) --
    def cmult_const(self, a, value, sigma):
        return self._unary(_lib.hetal_cmult_const, a, a.level, ctypes.byref(a._struct()), float(value), float(sigma))

    def add_const(self, a, value):
        return self._unary(_lib.hetal_add_const, a, a.level, ctypes.byref(a._struct()), float(value))

    def add_plain(self, a, pt):
        return self._unary(_lib.hetal_add_plain, a, a.level, ctypes.byref(a._struct()), ctypes.byref(pt._struct()))

    def refresh(self, sk, ct, a, e, scale=0.0):
        """The key holder's re-encryption at the top level (scale 0 keeps the scale)."""
        a, ap = _u64(a)
        e, ep = _i64(e)
        assert a.shape == (self.num_q, self.n) and e.shape == (self.n,)
        return self._unary(_lib.hetal_refresh, ct, self.max_level, sk._h, ctypes.byref(ct._struct()),
                           float(scale), ap, ep)

    def refresher(self, sk, randomness, scale=2.0 ** 40):
        """A refresh callback for the deep pipelines: the key holder re-encrypts in place (hetal_refresh) at
        `scale`, with randomness(i) -> (a, e) for the i-th call.  Keep the returned object alive while the
        pipeline runs."""
        count = [0]

        def cb(_user, ct_ptr):
            try:
                a, e = randomness(count[0])
                count[0] += 1
                a, ap = _u64(a)
                e, ep = _i64(e)
                return _lib.hetal_refresh(self._h, sk._h, ct_ptr, float(scale), ap, ep, ct_ptr)
            except Exception:  # the library turns a failed refresh into an error of the pipeline
                return -1
        fn = REFRESH_FN(cb)
        fn.calls = count
        return fn

    def poly_eval(self, keys, ct, coeffs, refresh=None):
        co, cp = _dbl(coeffs)
        out = self.new_ct(self.max_level)
        s = out._struct()
        _check(_lib.hetal_poly_eval(self._h, keys._h, ctypes.byref(ct._struct()), cp, len(co) - 1,
                                    refresh if refresh is not None else REFRESH_FN(), None, ctypes.byref(s)))
        out.level, out.scale = s.level, s.scale
        return out

    def softmax_rot_steps(self, c, s0):
        n = ctypes.c_int(0)
        _check(_lib.hetal_softmax_rot_steps(self._h, int(c), int(s0), None, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(_lib.hetal_softmax_rot_steps(self._h, int(c), int(s0), out.ctypes.data_as(_i32p), ctypes.byref(n)))
        return [int(x) for x in out[:n.value]]

    def softmax_approx(self, keys, m, c, params=None, refresh=None):
        """ASoftmax of a horizontally tiled a x c matrix -> (matrix, number of refreshes)."""
        p = softmax_default_params() if params is None else params
        out = Matrix(self, m.n_rb * self.ct_words(self.max_level), m.s0, 0, 0.0)
        s = out._struct()
        nref = ctypes.c_int(0)
        _check(_lib.hetal_softmax_approx(self._h, keys._h, ctypes.byref(m._struct()), int(c), ctypes.byref(p),
                                         refresh if refresh is not None else REFRESH_FN(), None, ctypes.byref(s),
                                         ctypes.byref(nref)))
        out._update(s)
        return out, nref.value

    def nag_step(self, keys, x, y, w, v, c, lr, gamma, params=None, refresh=None):
        """One NAG step of the encrypted training loop -> (W_{t+1}, V_{t+1}, number of refreshes)."""
        p = softmax_default_params() if params is None else params
        words = x.n_cb * self.ct_words(self.max_level)
        wo = Matrix(self, words, x.s0, 0, 0.0)
        vo = Matrix(self, words, x.s0, 0, 0.0)
        sw, sv = wo._struct(), vo._struct()
        nref = ctypes.c_int(0)
        _check(_lib.hetal_nag_step(self._h, keys._h, ctypes.byref(x._struct()), ctypes.byref(y._struct()),
                                   ctypes.byref(w._struct()), ctypes.byref(v._struct()), int(c), float(lr),
                                   float(gamma), ctypes.byref(p), refresh if refresh is not None else REFRESH_FN(),
                                   None, ctypes.byref(sw), ctypes.byref(sv), ctypes.byref(nref)))
        wo._update(sw)
        vo._update(sv)
        return wo, vo, nref.value

    def required_rot_steps(self, op, c, s0):
        n = ctypes.c_int(0)
        _check(_lib.hetal_required_rot_steps(self._h, int(op), int(c), int(s0), None, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(_lib.hetal_required_rot_steps(self._h, int(op), int(c), int(s0), out.ctypes.data_as(_i32p),
                                             ctypes.byref(n)))
        return [int(x) for x in out[:n.value]]


class Graph:
    """A recorded batch of products (Context.enc_matmul_batch_graph); keeps what it reads and writes alive."""

    def __init__(self, ctx, h, keep):
        self.ctx, self._h, self._keep = ctx, h, keep

    def launch(self):
        _check(_lib.hetal_graph_launch(self._h))

    def __del__(self, _destroy=_lib.hetal_graph_destroy):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)


class SecretKey:
    def __init__(self, ctx, s, sp, seed=None):
        self.ctx = ctx
        h = _vp()
        if seed is None:
            _check(_lib.hetal_sk_create(ctx._h, sp, ctypes.byref(h)))
        else:
            _check(_lib.hetal_keygen(ctx._h, int(seed), ctypes.byref(h)))
        self._h = h

    def __del__(self, _destroy=_lib.hetal_sk_destroy):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)


class KeySet:
    def __init__(self, ctx):
        self.ctx = ctx
        h = _vp()
        _check(_lib.hetal_keys_create(ctx._h, ctypes.byref(h)))
        self._h = h
        self.galois = set()

    def __del__(self, _destroy=_lib.hetal_keys_destroy):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            _destroy(h)

    def gen_relin(self, sk, a, e):
        a, ap = _u64(a)
        e, ep = _i64(e)
        c = self.ctx
        assert a.shape == (c.dnum, c.num_primes, c.n) and e.shape == (c.dnum, c.n)
        _check(_lib.hetal_keys_gen_relin(c._h, self._h, sk._h, ap, ep))

    def gen_galois(self, sk, g, a, e):
        a, ap = _u64(a)
        e, ep = _i64(e)
        c = self.ctx
        assert a.shape == (c.dnum, c.num_primes, c.n) and e.shape == (c.dnum, c.n)
        _check(_lib.hetal_keys_gen_galois(c._h, self._h, sk._h, int(g), ap, ep))
        self.galois.add(int(g))

    def gen_evk(self, sk, seed, rot_steps=(), conj=False, relin=False):
        """The relinearisation, rotation and conjugation keys with the library's randomness from `seed`."""
        c = self.ctx
        steps = (ctypes.c_int32 * max(1, len(rot_steps)))(*[int(r) for r in rot_steps])
        _check(_lib.hetal_gen_evk(c._h, self._h, sk._h, int(seed), steps, len(rot_steps), int(bool(conj)),
                                  int(bool(relin))))
        for r in rot_steps:
            if c.galois_rot(r) != 1:
                self.galois.add(c.galois_rot(r))
        if conj:
            self.galois.add(c.galois_conj())
