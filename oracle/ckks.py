"""CPU oracle: RNS-CKKS on residue arrays in coefficient form.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU library is checked against; only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library.

Representation.  A polynomial at level l is a uint64 array of shape
[l+1, N]: row i holds the coefficients modulo prime q_i, each in [0, q_i).
A ciphertext is a pair (c0, c1), stored as [2, l+1, N], with an FP64 scale.
Everything is kept in coefficient form; products go through the NTT of the C
core (``orc_polymul_limbs``) or, inside key switching, are accumulated in the
NTT domain and transformed back once (linearity of the transform).

What each operation computes (the CKKS operations of Sec. 2.2 of the paper on
the RNS variant of Sec. 5.1, in the textbook form):
  encode     m = round(scale * sigma^-1(z)), slot k <-> evaluation at zeta^(5^k)
  encrypt    (c0, c1) = (-a*s + m + e, a)            (secret-key form)
  decrypt    m = c0 + c1*s
  add/sub    limb-wise
  cmult      (c0*m, c1*m), scale multiplies
  mult       tensor (d0, d1, d2) then relinearise d2 with the key for s^2
  rotate     automorphism tau_g, g = 5^r (left rotation by r), key switched
  conjugate  automorphism g = 2N-1, key switched
  rescale    c_i <- (c_i - [c_l]_centred) * q_l^-1 mod q_i, top limb dropped
  mod_drop   top limbs dropped, scale unchanged
  mul_i      multiplication by X^(N/2), i.e. by i in every slot

Key switching (hybrid, dnum digits of alpha primes).  For d at level l with
primes q_0..q_l and special primes p_0..p_{K-1} (product P):
  ModUp_j(d): the residues of digit j's primes are kept; every other prime t
     of q_0..q_l, p_0..p_{K-1} receives the fast basis conversion
     sum_i [d_i (D_j/d_i)^-1]_{d_i} (D_j/d_i) mod t  (no overflow correction);
  the automorphism is applied to each extended digit after ModUp;
  (u0, u1) = sum_j tau_g(ModUp_j(d)) * (b_j, a_j) modulo P*Q_l;
  ModDown(u)_i = (u_i - conv_{P->q_i}(u_P)) * P^-1 mod q_i, where conv is the
     centred conversion (y_k taken in (-p_k/2, p_k/2]), so the division by P
     rounds and its error is zero-mean; the uncentred one leaves a mean error
     near (K+1)/2 per coefficient, which the slots next to +-1 amplify by ~N.
The key for s' is ksk_j = (-a_j s + e_j + g_j s', a_j) over all primes, with
g_j = P mod q_i when q_i lies in digit j, and 0 otherwise (0 modulo every p_k).

Parameters (the paper fixes N = 2^16 but not its primes): q_0 is the largest
prime below 2^q0_bits, q_1..q_L the largest primes below 2^q_bits in
descending order, p_0..p_{K-1} the largest primes below q_0; all are
1 mod 2N.  Digit j holds q_{alpha j} .. q_{alpha j + alpha - 1}.

Parity status: pinned (tests/test_oracle_*.py).
"""
import math

import numpy as np

from . import _native as nat

LIB = nat.LIB


class LevelError(RuntimeError):
    """Raised when an operation would need a level below 0."""


class KeyError_(RuntimeError):
    """Raised when a rotation key that an operation needs was not generated."""


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------

def primes_below(bound, m, count):
    out = np.zeros(count, dtype=np.uint64)
    got = LIB.orc_primes_below(int(bound), int(m), int(count), nat.u64ptr(out))
    if got != count:
        raise ValueError("not enough primes")
    return [int(x) for x in out]


class Params:
    def __init__(self, log_n, num_q, num_p, dnum, q0_bits=50, q_bits=40, scale_bits=40):
        self.log_n = log_n
        self.n = 1 << log_n
        self.slots = self.n // 2
        m = 2 * self.n
        q0 = primes_below(1 << q0_bits, m, 1)[0]
        rest = primes_below(1 << q_bits, m, num_q - 1) if num_q > 1 else []
        self.q = [q0] + rest
        self.p = primes_below(q0, m, num_p)
        self.num_q, self.num_p, self.dnum = num_q, num_p, dnum
        self.alpha = -(-num_q // dnum)
        self.max_level = num_q - 1
        self.scale = float(2 ** scale_bits)
        self.all_primes = self.q + self.p
        P = 1
        for p in self.p:
            P *= p
        self.P = P

    def digits(self, level):
        """Limb indices of each non-empty digit at `level`."""
        l = level + 1
        out = []
        for j in range(self.dnum):
            d = [i for i in range(j * self.alpha, (j + 1) * self.alpha) if i < l]
            if d:
                out.append(d)
        return out

    def galois_rot(self, r):
        """Galois element of a left rotation by r slots: 5^r mod 2N."""
        return pow(5, r % (self.n // 2), 2 * self.n)

    @property
    def galois_conj(self):
        return 2 * self.n - 1


PRESETS = {
    # 2^12 ring, q_0 (50-bit) + 4 x 40-bit, one special prime, one prime per digit.
    "toy": dict(log_n=12, num_q=5, num_p=1, dnum=5),
    # 2^16 ring, q_0 (50-bit) + 11 x 40-bit, three special primes, dnum = 4.
    "n16l12": dict(log_n=16, num_q=12, num_p=3, dnum=4),
    # 2^12 ring with the 2^16 ring's moduli chain shape (deep pipelines at test sizes).
    "n12l12": dict(log_n=12, num_q=12, num_p=3, dnum=4),
}


def preset(name):
    return Params(**PRESETS[name])


# --------------------------------------------------------------------------
# Limb-wise arithmetic helpers (coefficient form unless stated otherwise)
# --------------------------------------------------------------------------

def _qcol(qs):
    return np.asarray(qs, dtype=np.uint64)[:, None]


def add(a, b, qs):
    return (a + b) % _qcol(qs)


def sub(a, b, qs):
    return (a + (_qcol(qs) - b)) % _qcol(qs)


def neg(a, qs):
    return (_qcol(qs) - a) % _qcol(qs)


def polymul(a, b, qs, log_n):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    LIB.orc_polymul_limbs(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(out), a.shape[0], log_n, nat.u64ptr(nat.qarr(qs)))
    return out


def pointwise(a, b, qs, log_n):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    LIB.orc_mul_limbs(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(out), a.shape[0], log_n, nat.u64ptr(nat.qarr(qs)))
    return out


def mul_scalar(a, scalars, qs, log_n):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    LIB.orc_mul_scalar_limbs(nat.u64ptr(a), nat.u64ptr(nat.qarr(scalars)), nat.u64ptr(out), a.shape[0], log_n,
                             nat.u64ptr(nat.qarr(qs)))
    return out


def ntt(a, qs, log_n):
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    LIB.orc_ntt_batch(nat.u64ptr(out), out.shape[0], log_n, nat.u64ptr(nat.qarr(qs)))
    return out


def intt(a, qs, log_n):
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    LIB.orc_intt_batch(nat.u64ptr(out), out.shape[0], log_n, nat.u64ptr(nat.qarr(qs)))
    return out


def automorphism(a, qs, log_n, g):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    LIB.orc_automorphism_limbs(nat.u64ptr(a), nat.u64ptr(out), a.shape[0], log_n, nat.u64ptr(nat.qarr(qs)), int(g))
    return out


def basis_convert(x, src, dst, log_n):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.empty((len(dst), 1 << log_n), dtype=np.uint64)
    LIB.orc_basis_convert(nat.u64ptr(x), nat.u64ptr(nat.qarr(src)), len(src), nat.u64ptr(nat.qarr(dst)), len(dst),
                          nat.u64ptr(out), log_n)
    return out


def basis_convert_centered(x, src, dst, log_n):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.empty((len(dst), 1 << log_n), dtype=np.uint64)
    LIB.orc_basis_convert_centered(nat.u64ptr(x), nat.u64ptr(nat.qarr(src)), len(src), nat.u64ptr(nat.qarr(dst)),
                                   len(dst), nat.u64ptr(out), log_n)
    return out


def reduce_signed(c, qs, log_n):
    c = np.ascontiguousarray(c, dtype=np.int64)
    out = np.empty((len(qs), 1 << log_n), dtype=np.uint64)
    LIB.orc_reduce_signed(nat.i64ptr(c), nat.u64ptr(out), len(qs), log_n, nat.u64ptr(nat.qarr(qs)))
    return out


def mul_monomial_half(a, qs, n):
    """a * X^(N/2) in Z_q[X]/(X^N+1): coefficient k moves to k + N/2, wrapping with a sign flip."""
    h = n // 2
    out = np.empty_like(a)
    out[:, h:] = a[:, :h]
    out[:, :h] = neg(a[:, h:], qs)
    return out


# --------------------------------------------------------------------------
# Plaintexts, ciphertexts, keys
# --------------------------------------------------------------------------

class Pt:
    def __init__(self, m, scale):
        self.m = m            # uint64 [l+1, N]
        self.scale = float(scale)

    @property
    def level(self):
        return self.m.shape[0] - 1


class Ct:
    def __init__(self, c, scale):
        self.c = c            # uint64 [2, l+1, N]
        self.scale = float(scale)

    @property
    def level(self):
        return self.c.shape[1] - 1

    def copy(self):
        return Ct(self.c.copy(), self.scale)


class SecretKey:
    def __init__(self, prm, s_coeffs):
        s_coeffs = np.asarray(s_coeffs, dtype=np.int64)
        assert s_coeffs.shape == (prm.n,) and np.all(np.abs(s_coeffs) <= 1)
        self.coeffs = s_coeffs
        self.limbs = reduce_signed(s_coeffs, prm.all_primes, prm.log_n)   # [L+1+K, N]


class SwitchKey:
    """Key-switching key ksk_j = (b_j, a_j), j < dnum, over all L+1+K primes (coefficient form)."""

    def __init__(self, b, a, prm):
        self.b, self.a = b, a          # uint64 [dnum, L+1+K, N]
        self._ntt = {}
        self.prm = prm

    def ntt_rows(self, j, rows):
        """NTT form of (b_j, a_j) on the given prime rows (cached: keys are constants)."""
        key = (j, tuple(rows))
        if key not in self._ntt:
            qs = [self.prm.all_primes[r] for r in rows]
            self._ntt[key] = (ntt(self.b[j][rows], qs, self.prm.log_n), ntt(self.a[j][rows], qs, self.prm.log_n))
        return self._ntt[key]


def gen_switch_key(prm, sk, s_prime_limbs, a_rand, e_rand):
    """ksk_j = (-a_j s + e_j + g_j s', a_j) for j < dnum.

    a_rand: uint64 [dnum, L+1+K, N], uniform modulo each prime, coefficient form.
    e_rand: int64 [dnum, N], small signed error coefficients (shared by all primes).
    """
    allq = prm.all_primes
    nq = prm.num_q
    a_rand = np.ascontiguousarray(a_rand, dtype=np.uint64)
    assert a_rand.shape == (prm.dnum, len(allq), prm.n)
    b_all = np.empty_like(a_rand)
    for j in range(prm.dnum):
        e = reduce_signed(e_rand[j], allq, prm.log_n)
        b = add(neg(polymul(a_rand[j], sk.limbs, allq, prm.log_n), allq), e, allq)
        digit = [i for i in range(j * prm.alpha, (j + 1) * prm.alpha) if i < nq]
        for i in digit:
            p_mod = prm.P % allq[i]
            gs = mul_scalar(s_prime_limbs[i:i + 1], [p_mod], [allq[i]], prm.log_n)
            b[i] = add(b[i:i + 1], gs, [allq[i]])[0]
        b_all[j] = b
    return SwitchKey(b_all, a_rand.copy(), prm)


# --------------------------------------------------------------------------
# Encoding
# --------------------------------------------------------------------------

def encode_int(prm, z, scale):
    """round(scale * sigma^-1(z)) as N signed coefficients (z: N/2 complex slots)."""
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (prm.slots,)
    re = np.ascontiguousarray(z.real, dtype=np.float64)
    im = np.ascontiguousarray(z.imag, dtype=np.float64)
    out = np.empty(prm.n, dtype=np.int64)
    rc = LIB.orc_encode(nat.dblptr(re), nat.dblptr(im), prm.log_n, float(scale), nat.i64ptr(out))
    if rc != 0:
        raise OverflowError("encoded coefficient does not fit in 62 bits")
    return out


def encode(prm, z, level, scale):
    m = encode_int(prm, z, scale)
    return Pt(reduce_signed(m, prm.q[:level + 1], prm.log_n), scale)


def decode(prm, pt):
    """Slots of a plaintext: centred CRT of the first (up to) two limbs, then the
    evaluations m(zeta^(5^k)), computed as a size-2N DFT of the coefficients."""
    m = np.ascontiguousarray(pt.m, dtype=np.uint64)
    cnt = min(2, m.shape[0])
    coeffs = np.empty(prm.n, dtype=np.float64)
    LIB.orc_crt_centered(nat.u64ptr(m), cnt, prm.log_n, nat.u64ptr(nat.qarr(prm.q[:cnt])), nat.dblptr(coeffs))
    big_m = 2 * prm.n
    padded = np.zeros(big_m, dtype=np.float64)
    padded[:prm.n] = coeffs
    evals = np.fft.ifft(padded) * big_m          # evals[e] = sum_j m_j exp(2 pi i e j / 2N)
    idx = np.array([pow(5, k, big_m) for k in range(prm.slots)], dtype=np.int64)
    return evals[idx] / pt.scale


# --------------------------------------------------------------------------
# Encryption
# --------------------------------------------------------------------------

def encrypt(prm, sk, pt, a_rand, e_rand):
    """(c0, c1) = (-a*s + m + e, a); a_rand uint64 [l+1, N], e_rand int64 [N]."""
    l = pt.level + 1
    qs = prm.q[:l]
    a = np.ascontiguousarray(a_rand, dtype=np.uint64)
    assert a.shape == (l, prm.n)
    e = reduce_signed(e_rand, qs, prm.log_n)
    c0 = add(add(neg(polymul(a, sk.limbs[:l], qs, prm.log_n), qs), pt.m, qs), e, qs)
    return Ct(np.stack([c0, a.copy()]), pt.scale)


def decrypt(prm, sk, ct):
    l = ct.level + 1
    qs = prm.q[:l]
    m = add(ct.c[0], polymul(ct.c[1], sk.limbs[:l], qs, prm.log_n), qs)
    return Pt(m, ct.scale)


def refresh(prm, sk, ct, a_rand, e_rand, scale=None):
    """A fresh encryption at the top level of the message of `ct`, made by the key holder:
    decrypt, lift the plaintext polynomial m from q_0 (centred; every other limb must agree,
    i.e. |m| < q_0 / 2), re-encode it at `scale` as round(m * (scale / ct.scale)) (ties to
    even; `scale` None keeps the scale and m), re-encrypt with the given randomness (a_rand
    over all ciphertext primes).  This stands in for bootstrapping, which this library does
    not provide: the server hands the ciphertext back to the client.  Re-encoding at a fixed
    scale stops the drift that chains of squarings give the scale (each doubles its log
    distance from the primes)."""
    pt = decrypt(prm, sk, ct)
    q0 = prm.q[0]
    m0 = pt.m[0].astype(np.int64)
    m0 = np.where(pt.m[0] > q0 // 2, m0 - np.int64(q0), m0)
    for i in range(1, pt.level + 1):
        if not np.array_equal(reduce_signed(m0, [prm.q[i]], prm.log_n)[0], pt.m[i]):
            raise OverflowError("message too large to lift from q_0")
    new_scale = ct.scale if scale is None else float(scale)
    if scale is not None:
        r = new_scale / ct.scale
        m0 = np.rint(m0.astype(np.float64) * r).astype(np.int64)
    return encrypt(prm, sk, Pt(reduce_signed(m0, prm.q, prm.log_n), new_scale), a_rand, e_rand)


# --------------------------------------------------------------------------
# Key switching
# --------------------------------------------------------------------------

def mod_up(prm, d, digit, level):
    """Extend digit `digit` (limb indices) of d to all primes q_0..q_level, p_0..p_{K-1}."""
    l = level + 1
    ext = prm.q[:l] + prm.p
    out = np.empty((len(ext), prm.n), dtype=np.uint64)
    others = [t for t in range(len(ext)) if t not in digit]
    out[digit] = d[digit]
    out[others] = basis_convert(d[digit], [prm.q[i] for i in digit], [ext[t] for t in others], prm.log_n)
    return out


def mod_down(prm, u, level):
    """(u_i - conv_{P->q_i}(u_P)) * P^-1 mod q_i for i <= level, with the centred conversion
    (the division by P rounds, and the error it leaves has zero mean)."""
    l = level + 1
    qs = prm.q[:l]
    conv = basis_convert_centered(u[l:], prm.p, qs, prm.log_n)
    p_inv = [LIB.orc_invmod(prm.P % q, q) for q in qs]
    return mul_scalar(sub(u[:l], conv, qs), p_inv, qs, prm.log_n)


def key_switch(prm, d, ksk, g):
    """Switch d (coefficient form, level = rows-1) with ksk, automorphism g applied after ModUp."""
    level = d.shape[0] - 1
    l = level + 1
    ext = prm.q[:l] + prm.p
    key_rows = list(range(l)) + [prm.num_q + k for k in range(prm.num_p)]
    acc0 = np.zeros((len(ext), prm.n), dtype=np.uint64)
    acc1 = np.zeros_like(acc0)
    for j, digit in enumerate(prm.digits(level)):
        dt = mod_up(prm, d, digit, level)
        if g != 1:
            dt = automorphism(dt, ext, prm.log_n, g)
        dtn = ntt(dt, ext, prm.log_n)
        kb, ka = ksk.ntt_rows(j, key_rows)
        acc0 = add(acc0, pointwise(dtn, kb, ext, prm.log_n), ext)
        acc1 = add(acc1, pointwise(dtn, ka, ext, prm.log_n), ext)
    u0 = intt(acc0, ext, prm.log_n)
    u1 = intt(acc1, ext, prm.log_n)
    return mod_down(prm, u0, level), mod_down(prm, u1, level)


# --------------------------------------------------------------------------
# The evaluator: key material plus the homomorphic operations, with counters
# --------------------------------------------------------------------------

class Evaluator:
    def __init__(self, prm, sk=None):
        self.prm = prm
        self.sk = sk
        self.rot_keys = {}       # galois element -> SwitchKey
        self.relin_key = None
        self.counts = {}
        self._mask_cache = {}

    # -- key generation (randomness supplied by the caller) --
    def gen_relin_key(self, a_rand, e_rand):
        prm = self.prm
        s2 = polymul(self.sk.limbs, self.sk.limbs, prm.all_primes, prm.log_n)
        self.relin_key = gen_switch_key(prm, self.sk, s2, a_rand, e_rand)

    def gen_galois_key(self, g, a_rand, e_rand):
        prm = self.prm
        sg = automorphism(self.sk.limbs, prm.all_primes, prm.log_n, g)
        self.rot_keys[g] = gen_switch_key(prm, self.sk, sg, a_rand, e_rand)

    def _count(self, name, k=1):
        self.counts[name] = self.counts.get(name, 0) + k

    def reset_counts(self):
        self.counts = {}

    # -- level of a ciphertext --
    @staticmethod
    def level(ct):
        return ct.level

    # -- arithmetic --
    def _check_pair(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch %d vs %d" % (a.level, b.level))
        if abs(a.scale - b.scale) > 1e-9 * max(a.scale, b.scale):
            raise ValueError("scale mismatch %r vs %r" % (a.scale, b.scale))

    def add(self, a, b):
        self._check_pair(a, b)
        qs = self.prm.q[:a.level + 1]
        return Ct(np.stack([add(a.c[0], b.c[0], qs), add(a.c[1], b.c[1], qs)]), a.scale)

    def sub(self, a, b):
        self._check_pair(a, b)
        qs = self.prm.q[:a.level + 1]
        return Ct(np.stack([sub(a.c[0], b.c[0], qs), sub(a.c[1], b.c[1], qs)]), a.scale)

    def mul_i(self, a):
        qs = self.prm.q[:a.level + 1]
        return Ct(np.stack([mul_monomial_half(a.c[0], qs, self.prm.n), mul_monomial_half(a.c[1], qs, self.prm.n)]),
                  a.scale)

    def mod_drop(self, a, level):
        if level > a.level or level < 0:
            raise LevelError("cannot drop level %d to %d" % (a.level, level))
        return Ct(a.c[:, :level + 1].copy(), a.scale)

    def rescale(self, a):
        if a.level < 1:
            raise LevelError("no level left to rescale")
        self._count("rescale")
        prm = self.prm
        lv = a.level
        qt = prm.q[lv]
        qs = prm.q[:lv]
        out = np.empty((2, lv, prm.n), dtype=np.uint64)
        for p in range(2):
            top = a.c[p, lv].astype(np.int64)
            centred = np.where(a.c[p, lv] > qt // 2, top - np.int64(qt), top)
            r = reduce_signed(centred, qs, prm.log_n)
            inv = [LIB.orc_invmod(qt % q, q) for q in qs]
            out[p] = mul_scalar(sub(a.c[p, :lv], r, qs), inv, qs, prm.log_n)
        return Ct(out, a.scale / qt)

    def cmult(self, a, pt):
        if pt.level != a.level:
            raise ValueError("plaintext level %d vs ciphertext %d" % (pt.level, a.level))
        self._count("cmult")
        qs = self.prm.q[:a.level + 1]
        lg = self.prm.log_n
        return Ct(np.stack([polymul(a.c[0], pt.m, qs, lg), polymul(a.c[1], pt.m, qs, lg)]), a.scale * pt.scale)

    # -- constants (App. softmax evaluates real polynomials on ciphertexts) --
    def cmult_const(self, a, value, sigma):
        """Multiply by the real constant `value` encoded at scale `sigma`: the integer
        K = round(value * sigma) (ties to even) times both polynomials; the scale
        becomes scale * sigma.  No level is consumed (a rescale usually follows)."""
        k = round(float(value) * float(sigma))
        if abs(k) >= 1 << 62:
            raise OverflowError("constant does not fit in 62 bits")
        self._count("cmult_const")
        qs = self.prm.q[:a.level + 1]
        ks = [k % q for q in qs]
        lg = self.prm.log_n
        return Ct(np.stack([mul_scalar(a.c[0], ks, qs, lg), mul_scalar(a.c[1], ks, qs, lg)]),
                  a.scale * float(sigma))

    def add_const(self, a, value):
        """Add the real constant `value` to every slot: K = round(value * scale) is added to
        the constant coefficient of c0 (a constant polynomial decodes to K / scale in
        every slot)."""
        k = round(float(value) * a.scale)
        if abs(k) >= 1 << 62:
            raise OverflowError("constant does not fit in 62 bits")
        out = a.copy()
        for i, q in enumerate(self.prm.q[:a.level + 1]):
            out.c[0, i, 0] = np.uint64((int(out.c[0, i, 0]) + k) % q)
        return out

    def add_plain(self, a, values):
        """Add slot values encoded at the ciphertext's level and scale to c0."""
        pt = encode(self.prm, values, a.level, a.scale)
        qs = self.prm.q[:a.level + 1]
        return Ct(np.stack([add(a.c[0], pt.m, qs), a.c[1].copy()]), a.scale)

    def mask_plaintext(self, values, level):
        """A mask (slot values) encoded at `level` with scale q_level, so that
        cmult followed by rescale leaves the ciphertext scale unchanged."""
        values = np.asarray(values, dtype=np.complex128)
        key = (values.tobytes(), level)
        if key not in self._mask_cache:
            self._mask_cache[key] = encode(self.prm, values, level, float(self.prm.q[level]))
        return self._mask_cache[key]

    def cmult_mask(self, a, values):
        return self.cmult(a, self.mask_plaintext(values, a.level))

    def mult(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")
        if self.relin_key is None:
            raise KeyError_("relinearisation key missing")
        self._count("mult")
        self._count("keyswitch")
        prm = self.prm
        qs = prm.q[:a.level + 1]
        lg = prm.log_n
        d0 = polymul(a.c[0], b.c[0], qs, lg)
        d1 = add(polymul(a.c[0], b.c[1], qs, lg), polymul(a.c[1], b.c[0], qs, lg), qs)
        d2 = polymul(a.c[1], b.c[1], qs, lg)
        u0, u1 = key_switch(prm, d2, self.relin_key, 1)
        return Ct(np.stack([add(d0, u0, qs), add(d1, u1, qs)]), a.scale * b.scale)

    def _galois(self, a, g):
        if g not in self.rot_keys:
            raise KeyError_("no key for galois element %d" % g)
        self._count("keyswitch")
        prm = self.prm
        qs = prm.q[:a.level + 1]
        c0 = automorphism(a.c[0], qs, prm.log_n, g)
        u0, u1 = key_switch(prm, a.c[1], self.rot_keys[g], g)
        return Ct(np.stack([add(c0, u0, qs), u1]), a.scale)

    def rot(self, a, r):
        """Left rotation by r slots (r < 0: right rotation by -r)."""
        self._count("rot")
        return self._galois(a, self.prm.galois_rot(r))

    def conj(self, a):
        self._count("conj")
        return self._galois(a, self.prm.galois_conj)
