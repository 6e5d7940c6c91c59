"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no CKKS arithmetic: it only draws random numbers.  Every
random quantity the scheme consumes (secret key, key-switching key masks and
errors, encryption masks and errors) is drawn here and handed to both
implementations as an input, so that the two produce identical ciphertexts.

Streams are numpy PCG64 generators keyed by (seed, purpose, index...) through
SeedSequence, so each purpose has an independent, reproducible stream.

Distributions:
  secret      ternary with fixed Hamming weight h = 192: h positions drawn
              without replacement, each +1 or -1 (a sparse secret, as the
              security estimate the paper cites assumes); h = None gives a
              uniform ternary secret
  error       rounded normal, sigma = 3.2, clipped to [-19, 19] (6 sigma)
  uniform     uniform in [0, q) independently per prime (coefficient form)

Workload shapes stand in for the transfer-learning layers of the paper's
experiments (768-dimensional features from ViT-Base / MPNet, 2-100 classes):
features are N(0, 1) clipped to [-4, 4], weights uniform in [-0.05, 0.05].
"""
import zlib

import numpy as np

SIGMA = 3.2
ERROR_BOUND = 19

_PURPOSES = ("secret", "ksk_a", "ksk_e", "enc_a", "enc_e", "features", "weights", "labels", "toy", "slots", "logits",
             "refresh_a", "refresh_e")


def _rng(seed, purpose, *index):
    if purpose not in _PURPOSES:
        raise ValueError(purpose)
    tag = zlib.crc32(purpose.encode())
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), tag] + [int(i) for i in index])))


HAMMING_WEIGHT = 192


def ternary_secret(seed, n, hamming=HAMMING_WEIGHT):
    r = _rng(seed, "secret")
    if hamming is None:
        return r.integers(-1, 2, size=n, dtype=np.int64)
    s = np.zeros(n, dtype=np.int64)
    pos = r.choice(n, size=min(hamming, n), replace=False)
    s[pos] = r.choice(np.array([-1, 1], dtype=np.int64), size=len(pos))
    return s


def gaussian_error(rng, shape):
    e = np.rint(rng.normal(0.0, SIGMA, size=shape))
    return np.clip(e, -ERROR_BOUND, ERROR_BOUND).astype(np.int64)


def uniform_mod(rng, moduli, n):
    out = np.empty((len(moduli), n), dtype=np.uint64)
    for i, q in enumerate(moduli):
        out[i] = rng.integers(0, int(q), size=n, dtype=np.uint64)
    return out


def key_id(kind, galois=0):
    """Stable integer id of a key: kind 0 = relinearisation, 1 = Galois element `galois`."""
    return (int(kind) << 32) | int(galois)


def switch_key_randomness(seed, kid, dnum, all_moduli, n):
    """(a, e) of one key-switching key: a uint64 [dnum, len(all_moduli), n], e int64 [dnum, n]."""
    ra = _rng(seed, "ksk_a", kid)
    re = _rng(seed, "ksk_e", kid)
    a = np.stack([uniform_mod(ra, all_moduli, n) for _ in range(dnum)])
    e = np.stack([gaussian_error(re, n) for _ in range(dnum)])
    return a, e


def encryption_randomness(seed, index, moduli, n):
    """(a, e) of one encryption at the level given by `moduli`: a uint64 [l, n], e int64 [n]."""
    return uniform_mod(_rng(seed, "enc_a", index), moduli, n), gaussian_error(_rng(seed, "enc_e", index), n)


def refresh_randomness(seed, index, moduli, n):
    """(a, e) of the index-th re-encryption by the key holder (a over every ciphertext prime)."""
    return uniform_mod(_rng(seed, "refresh_a", index), moduli, n), gaussian_error(_rng(seed, "refresh_e", index), n)


def logits(seed, rows, cols, bound):
    """Softmax inputs: uniform in [-bound, bound] (the sampling of the softmax error table)."""
    return _rng(seed, "logits", rows, cols).uniform(-bound, bound, size=(rows, cols))


def features(seed, rows, cols):
    """Feature matrix: N(0, 1) clipped to [-4, 4]."""
    return np.clip(_rng(seed, "features", rows, cols).normal(size=(rows, cols)), -4.0, 4.0)


def weights(seed, rows, cols, bound=0.05):
    return _rng(seed, "weights", rows, cols).uniform(-bound, bound, size=(rows, cols))


def labels(seed, rows, classes):
    return _rng(seed, "labels", rows, classes).integers(0, classes, size=rows)


def toy_matrix(seed, rows, cols, index=0):
    """Entries uniform in [-1, 1]."""
    return _rng(seed, "toy", rows, cols, index).uniform(-1.0, 1.0, size=(rows, cols))


def slot_values(seed, count, index=0, bound=1.0, complex_=True):
    r = _rng(seed, "slots", count, index)
    re = r.uniform(-bound, bound, size=count)
    im = r.uniform(-bound, bound, size=count) if complex_ else np.zeros(count)
    return re + 1j * im


def softmax_minus_onehot(logits, labels_, classes):
    """P - Y for the gradient of softmax cross-entropy (plain FP64; builds the ATB input)."""
    z = logits - logits.max(axis=1, keepdims=True)
    p = np.exp(z)
    p /= p.sum(axis=1, keepdims=True)
    y = np.zeros_like(p)
    y[np.arange(len(labels_)), labels_] = 1.0
    return p - y
