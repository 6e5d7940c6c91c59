"""ctypes binding of the oracle's C core (``ckks_oracle.c``).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline may import the ``oracle`` package.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dblp = ctypes.POINTER(ctypes.c_double)


def build():
    """Compile the C core with gcc (plain -O2, OpenMP over limbs)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)


def _load():
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_powmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
        "orc_mulmod": (ctypes.c_uint64, [ctypes.c_uint64] * 3),
        "orc_invmod": (ctypes.c_uint64, [ctypes.c_uint64] * 2),
        "orc_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
        "orc_primes_below": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _u64p]),
        "orc_root_of_unity": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int]),
        "orc_ntt": (None, [_u64p, ctypes.c_int, ctypes.c_uint64]),
        "orc_intt": (None, [_u64p, ctypes.c_int, ctypes.c_uint64]),
        "orc_ntt_batch": (None, [_u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_intt_batch": (None, [_u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_polymul": (None, [_u64p, _u64p, _u64p, ctypes.c_int, ctypes.c_uint64]),
        "orc_polymul_limbs": (None, [_u64p, _u64p, _u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_polymul_schoolbook": (None, [_u64p, _u64p, _u64p, ctypes.c_int, ctypes.c_uint64]),
        "orc_mul_limbs": (None, [_u64p, _u64p, _u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_mul_scalar_limbs": (None, [_u64p, _u64p, _u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_automorphism": (None, [_u64p, _u64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]),
        "orc_automorphism_limbs": (None, [_u64p, _u64p, ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_uint64]),
        "orc_basis_convert": (None, [_u64p, _u64p, ctypes.c_int, _u64p, ctypes.c_int, _u64p, ctypes.c_int]),
        "orc_basis_convert_centered": (None, [_u64p, _u64p, ctypes.c_int, _u64p, ctypes.c_int, _u64p, ctypes.c_int]),
        "orc_dd_pi": (None, [_dblp]),
        "orc_dd_root_of_unity": (None, [ctypes.c_uint64, ctypes.c_uint64, _dblp]),
        "orc_encode": (ctypes.c_int, [_dblp, _dblp, ctypes.c_int, ctypes.c_double, _i64p]),
        "orc_reduce_signed": (None, [_i64p, _u64p, ctypes.c_int, ctypes.c_int, _u64p]),
        "orc_crt_centered": (None, [_u64p, ctypes.c_int, ctypes.c_int, _u64p, _dblp]),
        "orc_chacha20_quarter_round": (None, [_u32p]),
        "orc_chacha20_block": (None, [_u32p, ctypes.c_uint32, _u32p, _u32p]),
        "orc_stream_words": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_uint64, _u64p]),
        "orc_sample_uniform": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_int, _u64p]),
        "orc_sample_gaussian": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                       ctypes.c_int, ctypes.c_int, _i64p]),
        "orc_sample_ternary": (ctypes.c_int64, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_int, ctypes.c_int, _i64p]),
        "orc_set_threads": (None, [ctypes.c_int]),
        "orc_max_threads": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def u64ptr(a):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_u64p)


def i64ptr(a):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_i64p)


def u32ptr(a):
    assert a.dtype == np.uint32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u32p)


def dblptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dblp)


def qarr(qs):
    return np.ascontiguousarray(np.asarray(qs, dtype=np.uint64))
