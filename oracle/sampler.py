"""Oracle of the seeded sampling: the randomness of key generation and encryption drawn from a seed.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  The paper's client generates the secret key and the
public operation keys (Sec. 3.1) and encrypts; it does not say how randomness is drawn.  The reading this
library takes, written out here from its definitions:

  * generator: the ChaCha20 block function (RFC 8439) as a counter-based stream, key = the 64-bit seed,
    nonce = (purpose, index, sub), counter = block number (``ckks_oracle.c``: ``stream_word``);
  * purposes: SECRET = 1; KSK_A = 2 and KSK_E = 3 (index = the key's id: 0 for relinearisation, the Galois
    element g for a rotation or conjugation key; sub = digit * 64 + prime for KSK_A, the digit for KSK_E);
    ENC_A = 4 and ENC_E = 5 (index = the encryption's number; sub = the prime for ENC_A, 0 for ENC_E);
  * uniform residues modulo q by rejection (``orc_sample_uniform``), one stream per prime;
  * errors: the rounded Gaussian of standard deviation sigma = 3.2 on |x| <= 19 (6 sigma), by a cumulative
    table of 63-bit thresholds (``cdt_table``) and a sign bit, one value per coefficient shared by all primes;
  * the secret: ternary with exactly h = 192 nonzero coefficients (``orc_sample_ternary``).

Parity status: pinned.  ChaCha20 against the RFC's published block and quarter-round vectors and against
OpenSSL's implementation; the table recomputed in exact rational arithmetic with a rigorous bound on exp;
the samplers by chi-square tests of their histograms and by their exact invariants
(tests/test_oracle_sampler.py).
"""
import decimal

import numpy as np

from . import _native as nat

SECRET, KSK_A, KSK_E, ENC_A, ENC_E = 1, 2, 3, 4, 5
SIGMA = decimal.Decimal("3.2")
BOUND = 19
HAMMING_WEIGHT = 192


def cdt_table(sigma=SIGMA, bound=BOUND, prec=60):
    """Thresholds T_j = floor(2^63 F(j)), j < bound, of the rounded Gaussian on |x| <= bound: F(j) is the
    probability that |x| <= j, rho(i) = exp(-i^2 / (2 sigma^2)), P(|x| = 0) = rho(0) / S and P(|x| = i) =
    2 rho(i) / S for i >= 1, S = rho(0) + 2 sum_{i <= bound} rho(i).  Decimal arithmetic at `prec` digits; a
    threshold within 10^-30 of an integer would make the floor ambiguous and raises."""
    ctx = decimal.Context(prec=prec)
    two_s2 = ctx.multiply(2, ctx.multiply(sigma, sigma))
    rho = [ctx.exp(ctx.minus(ctx.divide(i * i, two_s2))) for i in range(bound + 1)]
    total = rho[0] + 2 * sum(rho[1:], decimal.Decimal(0))
    scale = decimal.Decimal(2) ** 63
    out, acc = [], rho[0]
    for j in range(bound):
        v = ctx.multiply(ctx.divide(acc, total), scale)
        f = int(v.to_integral_value(rounding=decimal.ROUND_FLOOR))
        frac = v - f
        if frac < decimal.Decimal("1e-30") or 1 - frac < decimal.Decimal("1e-30"):
            raise ArithmeticError("threshold %d too close to an integer" % j)
        out.append(f)
        acc = acc + 2 * rho[j + 1]
    return np.array(out, dtype=np.uint64)


_TABLE = None


def table():
    global _TABLE
    if _TABLE is None:
        _TABLE = cdt_table()
    return _TABLE


def stream_words(seed, purpose, index, sub, first, count):
    out = np.zeros(count, dtype=np.uint64)
    nat.LIB.orc_stream_words(seed, purpose, index, sub, first, count, nat.u64ptr(out))
    return out


def uniform(seed, purpose, index, sub, q, n):
    out = np.zeros(n, dtype=np.uint64)
    nat.LIB.orc_sample_uniform(seed, purpose, index, sub, int(q), n.bit_length() - 1, nat.u64ptr(out))
    return out


def gaussian(seed, purpose, index, sub, n):
    t = table()
    out = np.zeros(n, dtype=np.int64)
    nat.LIB.orc_sample_gaussian(seed, purpose, index, sub, nat.u64ptr(t), len(t), n.bit_length() - 1,
                                nat.i64ptr(out))
    return out


def ternary(seed, n, h=HAMMING_WEIGHT):
    out = np.zeros(n, dtype=np.int64)
    used = nat.LIB.orc_sample_ternary(seed, SECRET, 0, 0, h, n.bit_length() - 1, nat.i64ptr(out))
    if used < 0:
        raise ValueError("Hamming weight above N")
    return out


def key_id(galois=None):
    """0 for the relinearisation key, the Galois element for a rotation or conjugation key."""
    return 0 if galois is None else int(galois)


def switch_key_randomness(seed, kid, dnum, all_primes, n):
    """(a, e) of one switching key from the seed: a uint64 [dnum, len(all_primes), n], e int64 [dnum, n]."""
    a = np.stack([np.stack([uniform(seed, KSK_A, kid, j * 64 + t, q, n) for t, q in enumerate(all_primes)])
                  for j in range(dnum)])
    e = np.stack([gaussian(seed, KSK_E, kid, j, n) for j in range(dnum)])
    return a, e


def encryption_randomness(seed, index, moduli, n):
    """(a, e) of encryption number `index` at the level given by `moduli`: a uint64 [l, n], e int64 [n]."""
    a = np.stack([uniform(seed, ENC_A, index, i, q, n) for i, q in enumerate(moduli)])
    return a, gaussian(seed, ENC_E, index, 0, n)
