"""Pins of the oracle's encoder/decoder.

The encoder is checked against the direct definition of the inverse canonical
embedding evaluated in 60-digit decimal arithmetic (an O(N^2) sum, independent
of the double-double FFT), including the rounding rule; the slot order is pinned
by the textbook facts tau_{5^r} = cyclic left shift by r, tau_{-1} = conjugation.
"""
import decimal
from decimal import Decimal

import numpy as np
import pytest

from oracle import _native as nat
from oracle import ckks
from paper_2403_14111_amd import inputs

LIB = nat.LIB
decimal.getcontext().prec = 60


def dec_pi():
    """pi from Machin's formula, 16 atan(1/5) - 4 atan(1/239)."""
    def atan_inv(x):
        x = Decimal(x)
        total, term, k = Decimal(0), 1 / x, 0
        while abs(term) > Decimal(10) ** -58:
            total += term / (2 * k + 1) * (1 if k % 2 == 0 else -1)
            term /= x * x
            k += 1
        return total
    return 16 * atan_inv(5) - 4 * atan_inv(239)


PI = dec_pi()


def rounding_bound(prm, scale):
    """Slot error of rounding N coefficients (each off by at most 1/2): about sqrt(N)/2
    per slot for random signs; 8x that leaves a wide margin."""
    return 4.0 * np.sqrt(prm.n) / scale


def dec_cos_sin(x):
    c, s = Decimal(0), Decimal(0)
    term = Decimal(1)
    k = 0
    while abs(term) > Decimal(10) ** -58 or k < 4:
        if k % 2 == 0:
            c += term * (1 if (k // 2) % 2 == 0 else -1)
        else:
            s += term * (1 if (k // 2) % 2 == 0 else -1)
        k += 1
        term = term * x / k
    return c, s


def test_pi_double_double():
    out = np.empty(2)
    LIB.orc_dd_pi(nat.dblptr(out))
    assert abs(Decimal(out[0]) + Decimal(out[1]) - PI) < Decimal(10) ** -31


@pytest.mark.parametrize("j,m", [(1, 8192), (3, 8192), (2047, 8192), (2048, 8192), (5000, 8192), (131071, 131072),
                                 (40000, 131072)])
def test_dd_roots_of_unity(j, m):
    out = np.empty(4)
    LIB.orc_dd_root_of_unity(j, m, nat.dblptr(out))
    c, s = dec_cos_sin(2 * PI * j / m)
    assert abs(Decimal(out[0]) + Decimal(out[1]) - c) < Decimal(10) ** -30
    assert abs(Decimal(out[2]) + Decimal(out[3]) - s) < Decimal(10) ** -30


def round_rule(v):
    """Round half to even, with values within 2^-24 of a half-integer counted as ties."""
    f = v.to_integral_value(rounding=decimal.ROUND_FLOOR)
    frac = v - f
    f = int(f)
    if abs(frac - Decimal("0.5")) <= Decimal(2) ** -24:
        return f + (f & 1)
    return f + (1 if frac > Decimal("0.5") else 0)


def direct_encode(z, n, scale):
    """m_j = (2/N) Re sum_k z_k zeta^(-5^k j), zeta = exp(i pi / N), in decimal, then scaled and rounded."""
    m = 2 * n
    roots = [dec_cos_sin(2 * PI * e / m) for e in range(m)]
    exps = [pow(5, k, m) for k in range(n // 2)]
    out = []
    for j in range(n):
        acc = Decimal(0)
        for k, e in enumerate(exps):
            c, s = roots[(e * j) % m]
            # Re(z * (c - i s)) = re*c + im*s
            acc += Decimal(float(z[k].real)) * c + Decimal(float(z[k].imag)) * s
        out.append(round_rule(acc * 2 / n * Decimal(scale)))
    return out


def encode_c(z, log_n, scale):
    re = np.ascontiguousarray(np.real(z), dtype=np.float64)
    im = np.ascontiguousarray(np.imag(z), dtype=np.float64)
    out = np.empty(1 << log_n, dtype=np.int64)
    assert LIB.orc_encode(nat.dblptr(re), nat.dblptr(im), log_n, float(scale), nat.i64ptr(out)) == 0
    return [int(x) for x in out]


ODD_SCALE = 1099511562241  # an odd 40-bit scale, as masks use (q_l), to exercise exact half-integers


@pytest.mark.parametrize("log_n", [3, 4, 5])
@pytest.mark.parametrize("kind", ["random", "binary", "halves", "constant"])
@pytest.mark.parametrize("scale", [2.0 ** 40, float(ODD_SCALE), 3.0])
def test_encode_matches_direct_definition(log_n, kind, scale):
    n = 1 << log_n
    rng = np.random.default_rng(log_n * 7 + len(kind))
    if kind == "random":
        z = rng.uniform(-4, 4, n // 2) + 1j * rng.uniform(-4, 4, n // 2)
    elif kind == "binary":
        z = rng.integers(0, 2, n // 2).astype(float) + 0j
    elif kind == "halves":
        z = 0.5 * rng.integers(0, 2, n // 2) - 0.5j * rng.integers(0, 2, n // 2)
    else:
        z = np.ones(n // 2) + 0j
    assert encode_c(z, log_n, scale) == direct_encode(z, n, scale)


def test_encode_exact_ties_round_to_even():
    # z = 1 in every slot encodes to the constant polynomial scale * 1; with
    # z = 1/2 and an odd scale the constant coefficient is exactly x.5.
    log_n, n = 4, 16
    out = encode_c(np.full(n // 2, 0.5 + 0j), log_n, float(ODD_SCALE))
    half = ODD_SCALE // 2  # ODD_SCALE / 2 = half + 0.5
    assert out[0] == half + (half & 1) and all(v == 0 for v in out[1:])


@pytest.mark.parametrize("name", ["toy", "n16l12"])
def test_decode_inverts_encode(name):
    prm = ckks.preset(name)
    z = inputs.slot_values(1, prm.slots, bound=4.0)
    pt = ckks.encode(prm, z, 2, prm.scale)
    back = ckks.decode(prm, pt)
    assert np.max(np.abs(back - z)) < rounding_bound(prm, prm.scale)


@pytest.mark.parametrize("r", [1, 3, 100, 2047, -1, -64])
def test_slot_order_rotation_is_automorphism_5r(r):
    prm = ckks.preset("toy")
    z = inputs.slot_values(2, prm.slots)
    pt = ckks.encode(prm, z, 1, prm.scale)
    g = prm.galois_rot(r)
    rotated = ckks.Pt(ckks.automorphism(pt.m, prm.q[:2], prm.log_n, g), pt.scale)
    assert np.max(np.abs(ckks.decode(prm, rotated) - np.roll(z, -r))) < rounding_bound(prm, prm.scale)


def test_conjugation_is_automorphism_minus_one():
    prm = ckks.preset("toy")
    z = inputs.slot_values(3, prm.slots)
    pt = ckks.encode(prm, z, 1, prm.scale)
    conj = ckks.Pt(ckks.automorphism(pt.m, prm.q[:2], prm.log_n, prm.galois_conj), pt.scale)
    assert np.max(np.abs(ckks.decode(prm, conj) - np.conj(z))) < rounding_bound(prm, prm.scale)


def test_plaintext_product_is_slotwise_product():
    prm = ckks.preset("toy")
    z1 = inputs.slot_values(4, prm.slots)
    z2 = inputs.slot_values(5, prm.slots)
    p1 = ckks.encode(prm, z1, 1, 2.0 ** 30)
    p2 = ckks.encode(prm, z2, 1, 2.0 ** 30)
    prod = ckks.Pt(ckks.polymul(p1.m, p2.m, prm.q[:2], prm.log_n), 2.0 ** 60)
    assert np.max(np.abs(ckks.decode(prm, prod) - z1 * z2)) < 4 * rounding_bound(prm, 2.0 ** 30)


def test_mul_monomial_half_is_times_i():
    prm = ckks.preset("toy")
    z = inputs.slot_values(6, prm.slots)
    pt = ckks.encode(prm, z, 1, prm.scale)
    out = ckks.Pt(ckks.mul_monomial_half(pt.m, prm.q[:2], prm.n), pt.scale)
    assert np.max(np.abs(ckks.decode(prm, out) - 1j * z)) < rounding_bound(prm, prm.scale)
