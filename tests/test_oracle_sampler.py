"""The oracle's seeded sampler (oracle/sampler.py, ckks_oracle.c) against what fixes it independently: RFC 8439's
published ChaCha20 vectors and OpenSSL's implementation, the cumulative Gaussian table recomputed in exact
rational arithmetic with a rigorous bound on exp, chi-square tests of every distribution, and the exact
invariants of the secret.  The library's own sampler code that runs on the host (the table, the secret) is
compared with the oracle here too; its device sampler is compared on the GPU (tests/test_gpu_sampler.py)."""
import json
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import _native as nat
from oracle import sampler as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def block_bytes(key_bytes, nonce_bytes, counter):
    key = np.frombuffer(key_bytes, dtype="<u4").astype(np.uint32).copy()
    nonce = np.frombuffer(nonce_bytes, dtype="<u4").astype(np.uint32).copy()
    out = np.zeros(16, dtype=np.uint32)
    nat.LIB.orc_chacha20_block(nat.u32ptr(key), counter, nat.u32ptr(nonce), nat.u32ptr(out))
    return out.astype("<u4").tobytes()


def test_chacha20_rfc8439_vectors():
    g = json.load(open(os.path.join(GOLDEN, "chacha20_rfc8439.json")))
    x = np.array([int(v, 16) for v in g["quarter_round"]["in"]], dtype=np.uint32)
    nat.LIB.orc_chacha20_quarter_round(nat.u32ptr(x))
    assert [int(v) for v in x] == [int(v, 16) for v in g["quarter_round"]["out"]]
    b = g["block"]
    assert block_bytes(bytes.fromhex(b["key"]), bytes.fromhex(b["nonce"]), b["counter"]).hex() == b["serialized"]


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl not available")
def test_chacha20_against_openssl():
    """OpenSSL's chacha20 takes a 16-byte IV: the 32-bit block counter (little endian) and the 96-bit nonce."""
    rng = np.random.default_rng(5)
    for _ in range(4):
        key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
        nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
        counter = int(rng.integers(0, 2 ** 31))
        iv = counter.to_bytes(4, "little") + nonce
        r = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()], input=b"\0" * 192,
                           capture_output=True, check=True)
        want = r.stdout
        got = b"".join(block_bytes(key, nonce, counter + i) for i in range(3))
        assert got == want


def test_stream_words_are_little_endian_block_words():
    seed, purpose, index, sub = 0x0123456789ABCDEF, 2, 77, 130
    words = sp.stream_words(seed, purpose, index, sub, 0, 24)
    key = (seed & 0xFFFFFFFF).to_bytes(4, "little") + (seed >> 32).to_bytes(4, "little") + bytes(24)
    nonce = b"".join(v.to_bytes(4, "little") for v in (purpose, index, sub))
    ks = b"".join(block_bytes(key, nonce, b) for b in range(3))
    assert [int(w) for w in words] == [int.from_bytes(ks[8 * p:8 * p + 8], "little") for p in range(24)]


def exp_enclosure(x, terms=100):
    """e^x for a rational x >= 0 between the Taylor sum S and S + x^K / K! / (1 - x / (K + 1)) (the tail is
    below a geometric series of ratio x / (K + 1))."""
    s, t = Fraction(0), Fraction(1)
    for k in range(terms):
        s += t
        t = t * x / (k + 1)
    assert x < terms + 1
    return s, s + t / (1 - x / (terms + 1))


def test_gaussian_table_recomputed_exactly():
    """T_j = floor(2^63 F(j)) with F the cumulative probability of |x| <= j, rho(i) = exp(-i^2 / (2 sigma^2)),
    sigma = 16/5: every rho enclosed in rationals, F enclosed by monotonicity, and both ends of the enclosure
    give the table's value."""
    rho = []
    for i in range(20):
        lo, hi = exp_enclosure(Fraction(25 * i * i, 512))
        rho.append((1 / hi, 1 / lo))
    scale = 2 ** 63
    want = []
    for j in range(19):
        a_lo = rho[0][0] + 2 * sum(r[0] for r in rho[1:j + 1])
        a_hi = rho[0][1] + 2 * sum(r[1] for r in rho[1:j + 1])
        b_lo = 2 * sum(r[0] for r in rho[j + 1:])
        b_hi = 2 * sum(r[1] for r in rho[j + 1:])
        f_lo, f_hi = a_lo / (a_lo + b_hi), a_hi / (a_hi + b_lo)
        t_lo, t_hi = (f_lo * scale).__floor__(), (f_hi * scale).__floor__()
        assert t_lo == t_hi
        want.append(t_lo)
    assert [int(v) for v in sp.table()] == want
    assert all(a < b for a, b in zip(want, want[1:]))


def test_library_host_sampling_equals_the_oracle():
    """The library's host code (no GPU involved): its double-double table, and the secret of a seed."""
    from paper_2403_14111_amd import hetal
    assert np.array_equal(hetal.gaussian_table(), sp.table())
    for log_n, seed in ((12, 7), (16, 2000), (12, 2 ** 63 + 5)):
        assert np.array_equal(hetal.sample_ternary(log_n, seed, 192), sp.ternary(seed, 1 << log_n))


def test_secret_invariants():
    for seed in range(20):
        s = sp.ternary(seed, 1 << 12)
        assert np.count_nonzero(s) == 192 and set(np.unique(s)) <= {-1, 0, 1}
    signs = np.concatenate([sp.ternary(seed, 1 << 12)[sp.ternary(seed, 1 << 12) != 0] for seed in range(50)])
    assert stats.binomtest(int((signs > 0).sum()), len(signs)).pvalue > 1e-6
    counts = np.zeros(64)
    for seed in range(100):
        counts += np.bincount(np.nonzero(sp.ternary(seed, 1 << 12))[0] // 64, minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-6
    with pytest.raises(ValueError):
        sp.ternary(1, 1 << 12, h=5000)


def test_uniform_rejection_follows_its_definition():
    """Coefficient k takes the first of the words k, N + k, 2N + k, ... below floor(2^64 / q) q: checked word for
    word at a modulus just above 2^63, where about half of the words are rejected (some more than once)."""
    q, n = (1 << 63) + 12345, 1 << 12
    assert sp.uniform(0, 0, 0, 0, 3, 1 << 12).max() <= 2
    vals = sp.uniform(11, sp.KSK_A, 5, 3, q, n)
    bound = (2 ** 64 // q) * q
    layer0 = sp.stream_words(11, sp.KSK_A, 5, 3, 0, n)
    rejected = np.nonzero(layer0 >= np.uint64(bound))[0]
    assert len(rejected) >= 1
    ok = layer0 < np.uint64(bound)
    assert np.array_equal(vals[ok], layer0[ok] % np.uint64(q))
    for k in rejected:
        p = int(k)
        while True:
            p += n
            w = int(sp.stream_words(11, sp.KSK_A, 5, 3, p, 1)[0])
            if w < bound:
                break
        assert int(vals[k]) == w % q


def test_uniform_distribution():
    q = 40961
    counts = np.zeros(64)
    for seed in range(4):
        v = sp.uniform(seed, sp.ENC_A, seed, 0, q, 1 << 16)
        assert v.max() < q
        counts += np.bincount((v.astype(np.int64) * 64) // q, minlength=64)
    expected = np.array([((b + 1) * q + 63) // 64 - (b * q + 63) // 64 for b in range(64)], dtype=float)
    expected *= counts.sum() / expected.sum()
    assert stats.chisquare(counts, expected).pvalue > 1e-6


def test_gaussian_distribution():
    t = [int(v) for v in sp.table()] + [2 ** 63]
    mag_p = np.array([t[0]] + [t[j] - t[j - 1] for j in range(1, 20)], dtype=float) / 2.0 ** 63
    p = np.zeros(39)
    p[19] = mag_p[0]
    for j in range(1, 20):
        p[19 + j] = p[19 - j] = mag_p[j] / 2
    # the table's distribution is the rounded Gaussian of sigma 3.2 to within 2^-62 per value
    rho = np.exp(-np.arange(-19, 20) ** 2 / (2 * 3.2 ** 2))
    assert np.abs(p - rho / rho.sum()).max() < 2.0 ** -50
    x = np.concatenate([sp.gaussian(seed, sp.KSK_E, 9, seed, 1 << 16) for seed in range(8)])
    assert np.abs(x).max() <= 19
    counts = np.bincount(x + 19, minlength=39).astype(float)
    exp = p * len(x)
    keep = exp >= 5
    obs = np.concatenate([counts[keep], [counts[~keep].sum()]])
    e = np.concatenate([exp[keep], [exp[~keep].sum()]])
    assert stats.chisquare(obs, e).pvalue > 1e-6
    assert abs(x.std() - 3.2) < 0.02


def test_randomness_shapes():
    a, e = sp.switch_key_randomness(3, sp.key_id(5), 2, [12289, 40961, 65537], 1 << 12)
    assert a.shape == (2, 3, 4096) and e.shape == (2, 4096)
    assert np.array_equal(a[1, 2], sp.uniform(3, sp.KSK_A, 5, 64 + 2, 65537, 4096))
    a, e = sp.encryption_randomness(3, 9, [12289, 40961], 1 << 12)
    assert a.shape == (2, 4096) and np.array_equal(e, sp.gaussian(3, sp.ENC_E, 9, 0, 4096))
