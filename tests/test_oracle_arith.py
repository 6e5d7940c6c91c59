"""Pins of the oracle's integer core against definitions computed independently in Python.

Each check targets a plausible slip: a wrong root or twist (NTT vs schoolbook),
a dropped wrap-around sign (negacyclic products, automorphisms), a wrong CRT
weight (basis conversion), a prime-search off-by-one (primes).
"""
import random

import numpy as np
import pytest

from oracle import _native as nat
from oracle import ckks

LIB = nat.LIB


def py_is_prime(n):
    """Miller-Rabin written independently of the C core (random and small bases)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    rnd = random.Random(n)
    for a in small + [rnd.randrange(2, n - 1) for _ in range(8)]:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def schoolbook_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] = (out[k] + a[i] * b[j]) % q
            else:
                out[k - n] = (out[k - n] - a[i] * b[j]) % q
    return out


@pytest.mark.parametrize("name", ["toy", "n16l12"])
def test_primes_follow_the_rule(name):
    prm = ckks.preset(name)
    m = 2 * prm.n
    for q in prm.all_primes:
        assert q % m == 1 and py_is_prime(q)
    assert len(set(prm.all_primes)) == len(prm.all_primes)
    # q_0: the largest such prime below 2^50 -- every candidate above it is composite
    for cand in range(prm.q[0] + m, 1 << 50, m):
        assert not py_is_prime(cand)
    # q_1.. descending, the largest below 2^40, no candidate skipped
    qs = prm.q[1:]
    assert qs == sorted(qs, reverse=True) and qs[0] < (1 << 40)
    cands = [c for c in range(qs[-1], 1 << 40, m) if py_is_prime(c)]
    assert sorted(cands, reverse=True) == qs
    # special primes: the largest below q_0
    ps = prm.p
    cands = [c for c in range(ps[-1], prm.q[0], m) if py_is_prime(c)]
    assert sorted(cands, reverse=True) == ps


def test_is_prime_agrees_on_a_range():
    for n in list(range(2, 3000)) + [(1 << 61) - 1, (1 << 50) - 27, 1000000007 * 998244353]:
        assert bool(LIB.orc_is_prime(n)) == py_is_prime(n), n


@pytest.mark.parametrize("log_n", [3, 4, 12, 16])
def test_root_of_unity_has_order_2n(log_n):
    q = ckks.primes_below(1 << 50, 2 << log_n, 1)[0]
    psi = LIB.orc_root_of_unity(q, log_n)
    n = 1 << log_n
    assert pow(psi, n, q) == q - 1 and pow(psi, 2 * n, q) == 1


@pytest.mark.parametrize("log_n", [2, 3, 5])
def test_ntt_is_evaluation_at_odd_powers(log_n):
    n = 1 << log_n
    q = ckks.primes_below(1 << 40, 2 * n, 1)[0]
    psi = LIB.orc_root_of_unity(q, log_n)
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    out = a.copy()
    LIB.orc_ntt(nat.u64ptr(out), log_n, q)
    for k in range(n):
        x = pow(psi, 2 * k + 1, q)
        assert int(out[k]) == sum(int(a[j]) * pow(x, j, q) for j in range(n)) % q


@pytest.mark.parametrize("log_n,bits", [(3, 40), (4, 50), (6, 50), (6, 40)])
def test_polymul_matches_python_schoolbook(log_n, bits):
    n = 1 << log_n
    q = ckks.primes_below(1 << bits, 2 * n, 1)[0]
    rng = np.random.default_rng(bits + log_n)
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    out = np.empty_like(a)
    LIB.orc_polymul(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(out), log_n, q)
    assert [int(x) for x in out] == schoolbook_negacyclic([int(x) for x in a], [int(x) for x in b], q)


@pytest.mark.parametrize("log_n", [8, 10])
def test_polymul_matches_c_schoolbook(log_n):
    n = 1 << log_n
    q = ckks.primes_below(1 << 50, 2 * n, 2)[1]
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)
    o1, o2 = np.empty_like(a), np.empty_like(a)
    LIB.orc_polymul(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(o1), log_n, q)
    LIB.orc_polymul_schoolbook(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(o2), log_n, q)
    assert np.array_equal(o1, o2)


def test_x_to_the_n_is_minus_one():
    log_n, n = 5, 32
    q = ckks.primes_below(1 << 40, 2 * n, 1)[0]
    a = np.zeros(n, dtype=np.uint64)
    a[n - 1] = 1   # X^(N-1)
    b = np.zeros(n, dtype=np.uint64)
    b[1] = 1       # X
    out = np.empty_like(a)
    LIB.orc_polymul(nat.u64ptr(a), nat.u64ptr(b), nat.u64ptr(out), log_n, q)
    expect = np.zeros(n, dtype=np.uint64)
    expect[0] = q - 1
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("log_n", [12, 16])
def test_ntt_round_trip(log_n):
    prm = ckks.preset("toy" if log_n == 12 else "n16l12")
    rng = np.random.default_rng(7)
    qs = prm.all_primes
    a = np.stack([rng.integers(0, q, size=prm.n, dtype=np.uint64) for q in qs])
    assert np.array_equal(ckks.intt(ckks.ntt(a, qs, log_n), qs, log_n), a)


def py_automorphism(a, g, q):
    n = len(a)
    out = [0] * n
    for j, v in enumerate(a):
        e = (g * j) % (2 * n)
        if e < n:
            out[e] = (out[e] + v) % q
        else:
            out[e - n] = (out[e - n] - v) % q
    return out


def test_automorphism_definition_and_laws():
    log_n, n = 6, 64
    q = ckks.primes_below(1 << 40, 2 * n, 1)[0]
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, size=n, dtype=np.uint64)
    b = rng.integers(0, q, size=n, dtype=np.uint64)

    def aut(x, g):
        out = np.empty_like(x)
        LIB.orc_automorphism(nat.u64ptr(np.ascontiguousarray(x)), nat.u64ptr(out), log_n, q, g)
        return out

    def mul(x, y):
        out = np.empty_like(x)
        LIB.orc_polymul(nat.u64ptr(np.ascontiguousarray(x)), nat.u64ptr(np.ascontiguousarray(y)), nat.u64ptr(out),
                        log_n, q)
        return out

    for g in (5, 25, 2 * n - 1, 3, 77):
        assert [int(x) for x in aut(a, g)] == py_automorphism([int(x) for x in a], g, q)
        # ring homomorphism
        assert np.array_equal(aut(mul(a, b), g), mul(aut(a, g), aut(b, g)))
    # composition: tau_g o tau_h = tau_{g h mod 2N}
    for g, h in [(5, 25), (5, 2 * n - 1), (125, 3)]:
        assert np.array_equal(aut(aut(a, h), g), aut(a, (g * h) % (2 * n)))
    # tau_{5^(N/2)} is the identity (5 has order N/2 modulo 2N)
    assert np.array_equal(aut(a, pow(5, n // 2, 2 * n)), a)


def test_basis_conversion_is_crt_lift_plus_multiple_of_d():
    log_n, n = 4, 16
    prm = ckks.preset("n16l12")
    src = prm.q[3:6]
    dst = prm.q[:3] + prm.p
    D = src[0] * src[1] * src[2]
    rng = np.random.default_rng(11)
    vals = [int(rng.integers(0, 1 << 62)) * int(rng.integers(0, 1 << 60)) % D for _ in range(n)]
    x = np.array([[v % s for v in vals] for s in src], dtype=np.uint64)
    out = ckks.basis_convert(x, src, dst, log_n)
    for k in range(n):
        # the lift is sum_i y_i (D/d_i) for y_i in [0, d_i): it equals vals[k] + u D with 0 <= u < len(src)
        lift = sum(((vals[k] % s) * pow(D // s, -1, s) % s) * (D // s) for s in src)
        u = (lift - vals[k]) // D
        assert (lift - vals[k]) % D == 0 and 0 <= u < len(src)
        for t, qt in enumerate(dst):
            assert int(out[t, k]) == lift % qt


def test_crt_centered():
    prm = ckks.preset("n16l12")
    q0, q1 = prm.q[0], prm.q[1]
    n = 16
    rng = np.random.default_rng(5)
    vals = [int(rng.integers(-(1 << 62), 1 << 62)) * int(rng.integers(1, 1 << 20)) for _ in range(n)]
    vals[0], vals[1] = (q0 * q1 - 1) // 2, -((q0 * q1 - 1) // 2)
    limbs = np.array([[v % q0 for v in vals], [v % q1 for v in vals]], dtype=np.uint64)
    out = np.empty(n)
    LIB.orc_crt_centered(nat.u64ptr(limbs), 2, 4, nat.u64ptr(nat.qarr([q0, q1])), nat.dblptr(out))
    assert np.array_equal(out, np.array([float(v) for v in vals]))


def test_reduce_signed():
    prm = ckks.preset("toy")
    c = np.array([0, 1, -1, 2 ** 61, -(2 ** 61), 12345678901234], dtype=np.int64)
    c = np.concatenate([c, np.zeros(prm.n - len(c), dtype=np.int64)])
    out = ckks.reduce_signed(c, prm.q, prm.log_n)
    for i, q in enumerate(prm.q):
        assert [int(x) for x in out[i, :6]] == [int(v) % q for v in c[:6]]
