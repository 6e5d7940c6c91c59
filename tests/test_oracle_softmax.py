"""Pins of the softmax oracle (App. softmax) against what the paper and the mathematics fix."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ckks
from oracle import matrix as mx
from oracle import softmax as sm
from paper_2403_14111_amd import inputs
from tests.oracle_setup import make_oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PV = np.polynomial.polynomial.polyval


def test_f_is_the_closed_form_comparison_polynomial():
    """f_3(x) = sum_{i<=3} 4^-i C(2i, i) x (1 - x^2)^i, the textbook sign-approximating polynomial
    whose coefficients the paper prints."""
    poly = [Fraction(0)] * 8
    for i in range(4):
        term = [Fraction(0), Fraction(1)]                      # x
        for _ in range(i):                                      # times (1 - x^2)
            nxt = [Fraction(0)] * (len(term) + 2)
            for k, v in enumerate(term):
                nxt[k] += v
                nxt[k + 2] -= v
            term = nxt
        w = Fraction(math.comb(2 * i, i), 4 ** i)
        for k, v in enumerate(term):
            poly[k] += w * v
    assert [Fraction(v, sm.F_DEN) for v in sm.F_NUM] == poly
    assert PV(1.0, sm.f_coeffs()) == 1.0 and PV(-1.0, sm.f_coeffs()) == -1.0


def test_g_and_the_composite_sign_approximation():
    x = np.linspace(-1, 1, 40001)
    g = PV(x, sm.g_coeffs())
    assert np.allclose(PV(-x, sm.g_coeffs()), -g)                # odd
    assert np.abs(g).max() <= 1.0                                # maps [-1, 1] into itself
    assert sm.g_coeffs()[1] == 4589 / 1024                       # slope at 0 above 1: it pushes away from 0
    y = x.copy()
    for _ in range(3):
        y = PV(y, sm.g_coeffs())
    fy = PV(y, sm.f_coeffs())
    assert np.abs(fy).max() <= 1.0                               # Acomp stays in [0, 1]: Amax <= max
    far = np.abs(x) >= 1 / 64
    assert np.abs(fy[far] - np.sign(x[far])).max() < 0.02
    assert PV(0.0, sm.comp_out_coeffs()) == 0.5                  # Acomp(a, a) = 1/2


def dep(x, prm):
    for i in range(prm.n - 1, -1, -1):
        x = PV(x, sm.dep_coeffs(prm, i))
    return x


def test_dep_maps_the_extended_domain_into_the_base_interval():
    prm = sm.SoftmaxParams()
    span = prm.L ** prm.n * prm.R
    x = np.linspace(-span, span, 200001)
    d = dep(x, prm)
    assert np.abs(d).max() <= prm.R
    # B alone: [-2R, 2R] -> [-R, R], with B(3R/2) = R (its maximum)
    b = PV(np.linspace(-2 * prm.R, 2 * prm.R, 10001), sm.dep_coeffs(prm, 0))
    assert np.abs(b).max() <= prm.R + 1e-12
    assert PV(1.5 * prm.R, sm.dep_coeffs(prm, 0)) == pytest.approx(prm.R, rel=1e-15)


def test_dep_lemmas_derivative_and_lower_bound():
    """0 <= D_n' <= 1 on [-r, r] and D_n(x) >= x - delta L^2 / (L^2 - 1) x^3 on [0, r] (the lemmas
    before the theorem), for B with delta = 4 / (27 R^2) and r = R."""
    prm = sm.SoftmaxParams()
    r = prm.R
    delta = 4.0 / (27.0 * r * r)
    x = np.linspace(-r, r, 20001)
    d = dep(x, prm)
    slope = np.diff(d) / np.diff(x)
    assert slope.min() >= 0.0 and slope.max() <= 1.0 + 1e-9
    xp = x[x >= 0]
    lower = xp - delta * prm.L ** 2 / (prm.L ** 2 - 1) * xp ** 3
    assert np.all(dep(xp, prm) >= lower - 1e-12)


def test_dep_correction_undoes_the_extension_near_zero():
    """B_inv(D_n(x)) is much closer to x than D_n(x) is: the reading of B_inv's sign."""
    prm = sm.SoftmaxParams()
    x = np.linspace(-2, 2, 4001)
    x = x[np.abs(x) > 0.05]
    d = dep(x, prm)
    back = PV(d, sm.dep_inv_coeffs(prm))
    assert (np.abs(back - x) / np.abs(d - x)).max() < 0.1
    printed = [-v if k in (3, 5) else v for k, v in enumerate(sm.dep_inv_coeffs(prm))]
    assert (np.abs(PV(d, printed) - x) / np.abs(d - x)).min() > 1.5   # the printed sign doubles the error


def test_aexp_and_ainv_accuracy():
    prm = sm.SoftmaxParams()
    x = np.linspace(-8, 8, 8001)
    assert np.abs(sm.aexp_plain(x, prm) / np.exp(x) - 1.0).max() < 1e-10
    y = np.linspace(1, 150, 8001)
    assert np.abs(sm.ainv_plain(y, prm) * y - 1.0).max() < 1e-12
    # p is the L^2 projection: the error of p(t) - e^t is orthogonal to 1, t, ..., t^12 on [-1, 1]
    t, w = np.polynomial.legendre.leggauss(40)
    p = PV(t * prm.exp_B, sm.exp_coeffs())
    for k in range(13):
        assert abs(np.sum(w * (p - np.exp(t)) * t ** k)) < 1e-14



def test_aexp_polynomial_equals_the_closed_form_legendre_series():
    """The L^2 projection of e^t onto degree <= 12 on [-1, 1] is the truncated Legendre series, whose coefficients have
    a closed form: int_{-1}^{1} e^t P_n(t) dt = 2 i_n(1), i_n the modified spherical Bessel function of the first kind,
    so p = sum_n (2n + 1) i_n(1) P_n.  Computed here with scipy's Bessel function, independently of the oracle's
    quadrature, and compared monomial by monomial after the oracle's 1/B scaling."""
    from scipy.special import spherical_in
    prm = sm.SoftmaxParams()
    leg = [(2 * n + 1) * spherical_in(n, 1.0) for n in range(prm.exp_degree + 1)]
    mono = np.polynomial.legendre.leg2poly(leg)
    want = [float(mono[k]) / float(prm.exp_B) ** k for k in range(prm.exp_degree + 1)]
    got = sm.exp_coeffs(prm.exp_degree, prm.exp_B)
    scale = max(abs(v) for v in want)
    for k in range(prm.exp_degree + 1):
        assert abs(got[k] - want[k]) <= 1e-13 * scale, k
    assert abs(leg[0] - np.sinh(1.0)) < 1e-15           # the mean of e^t on [-1, 1]


def test_ainv_equals_the_closed_form_of_goldschmidts_iteration():
    """Goldschmidt's iteration from y = x / R (a = 2 - y = 1 + b, b = 1 - y; b <- b^2, a <- a (1 + b)) keeps
    y a_k = 1 - b_0^(2^(k+1)) exactly, so after the 16 steps AInv(x) = (1 - (1 - x / R)^(2^17)) / x.  Near 0 the
    remainder is large and fixes the step count and the update order (one step fewer doubles b_0's exponent's
    distance from the truth); on [1, 150] it is 1/x."""
    prm = sm.SoftmaxParams()
    x = np.array([1e-3, 3e-3, 1e-2, 0.05, 0.5, 1.0, 7.0, 64.0, 150.0, 199.0])
    want = (1.0 - np.exp(2.0 ** (prm.inv_iters + 1) * np.log(np.abs(1.0 - x / prm.inv_R)))) / x  # even power
    got = sm.ainv_plain(x, prm)
    assert np.abs(got / want - 1.0).max() < 1e-10
    fewer = sm.ainv_plain(x[:2], sm.SoftmaxParams(inv_iters=prm.inv_iters - 1))
    assert np.abs(fewer / want[:2] - 1.0).min() > 0.1     # a dropped step would be caught


def test_stored_aexp_polynomial_is_the_oracles_projection():
    """tests/golden/aexp_coeffs.json, which both sides of the GPU parity tests take as input, holds the
    oracle's L^2 projection exactly (the file is regenerated by tests/golden/make_aexp_coeffs.py)."""
    from tests.golden_data import aexp_coeffs
    assert aexp_coeffs() == sm.exp_coeffs(12, 8)

def test_the_papers_example_is_covered():
    """(8, 10, 13): softmax (0.006, 0.047, 0.946) (main text), which the plain domain extension misses
    and normalisation first recovers."""
    x = np.array([[8.0, 10.0, 13.0]])
    assert np.round(sm.softmax_rows(x), 3).tolist() == [[0.006, 0.047, 0.946]]
    assert np.abs(sm.asoftmax_rows(x, sm.SoftmaxParams()) - sm.softmax_rows(x)).max() < 0.003


@pytest.mark.parametrize("c", [3, 10])
def test_theorem_bound_holds_per_input(c):
    """|Softmax(x) - p(D_n(x'))| < beta(c, delta, r, L) + eps with r = max - Amax of each input
    (Thm. softmaxbound; p is exact to 1e-10 here, see the accuracy test)."""
    prm = sm.SoftmaxParams(precise=False)
    X = inputs.logits(40 + c, 4000, c, 128.0)
    cp = mx.next_pow2(c)
    xs = np.full((len(X), cp), -0.5)
    xs[:, :c] = X / (2.0 * prm.r_max)
    m = sm.amax_plain(xs, prm) * (2.0 * prm.r_max)
    r = X.max(axis=1) - m
    assert np.all(r >= 0)                                        # Amax <= max
    err = np.abs(sm.asoftmax_rows(X, prm) - sm.softmax_rows(X)).max(axis=1)
    delta = 4.0 / (27.0 * prm.R ** 2)
    beta = np.array([sm.beta_bound(c, delta, max(ri, 1e-3), prm.L) for ri in r])
    assert np.all(err < beta + 1e-9)


def table_errors(c, R, prm, n, seed):
    mxe, tot, cnt = 0.0, 0.0, 0
    for k, r in enumerate((4, 8, 32, 128)):
        if r > R:
            break
        X = inputs.logits(seed + k, n, c, float(r))
        d = np.abs(sm.asoftmax_rows(X, prm) - sm.softmax_rows(X))
        mxe, tot, cnt = max(mxe, d.max()), tot + d.sum(), cnt + d.size
    return mxe, tot / cnt


def test_error_table():
    """Table softmaxerr, every cell of this method's three columns: sampled maximum within 2.5x of the
    printed maximum, mean within 1.5x of the printed mean, and the norm-only column no worse (this
    AExp is more accurate than the paper's)."""
    table = json.load(open(os.path.join(GOLDEN, "softmax_err_table.json")))
    cols = {"norm": sm.SoftmaxParams(extend=False, precise=False), "extn": sm.SoftmaxParams(precise=False),
            "prec": sm.SoftmaxParams()}
    for row in table["rows"]:
        for name, prm in cols.items():
            if name not in row:
                continue
            tmax, tavg = row[name]
            emax, eavg = table_errors(row["c"], row["R"], prm, 6000, 500 + row["c"] * 10 + row["R"])
            if name == "norm":
                assert emax <= tmax and eavg <= tavg, (row, name)
            else:
                assert emax <= 2.5 * tmax and eavg <= 1.5 * tavg, (row, name, emax, eavg)


def tiled_blocks(M, cp, s0, s1):
    a, c = M.shape
    P = np.zeros((a, cp))
    P[:, :c] = M
    return [b[0] for b in mx.block_encode(mx.tile_horizontal(P, s1), s0, s1)]


@pytest.mark.parametrize("c", [3, 10])
def test_block_algorithm_on_the_simulator_equals_the_row_form(c):
    """The slot-level algorithm (rotations, masks, tiling) computes the row-wise form, and leaves the
    output tiled horizontally with zeros in the padded classes."""
    prm_c = ckks.preset("n12l12")
    s0, s1 = 16, 128
    M = inputs.logits(60 + c, 20, c, 64.0)
    cp = mx.next_pow2(c)
    sim = sm.ScaledSim(prm_c)
    xs = [sim.encrypt(z, 8, prm_c.scale) for z in tiled_blocks(M, cp, s0, s1)]
    prm = sm.SoftmaxParams()
    out, nref = sm.asoftmax_blocks(sim, xs, c, s0, s1, prm, sm.exp_coeffs(), prm_c.q, prm_c.max_level, sim.refresh)
    assert nref > 0
    got = mx.block_decode([[o.z.real] for o in out], s0, s1)[:20]
    want = np.zeros((20, cp))
    want[:, :c] = sm.asoftmax_rows(M, prm)
    assert np.abs(got - np.tile(want, (1, s1 // cp))).max() < 1e-11
    assert np.abs(mx.block_decode([[o.z.imag] for o in out], s0, s1)).max() == 0.0


def test_block_algorithm_needs_refreshes_without_a_refresh_it_fails():
    prm_c = ckks.preset("n12l12")
    sim = sm.ScaledSim(prm_c)
    xs = [sim.encrypt(np.zeros(prm_c.slots), 11, prm_c.scale)]
    with pytest.raises(ckks.LevelError):
        sm.asoftmax_blocks(sim, xs, 10, 16, 128, sm.SoftmaxParams(), sm.exp_coeffs(), prm_c.q, prm_c.max_level)


def test_refresh_keeps_the_message_and_scale():
    ev = make_oracle("toy", seed=77, relin=False, conj=False)
    prm = ev.prm
    z = inputs.slot_values(5, prm.slots, bound=3.0)
    pt = ckks.encode(prm, z, 1, prm.scale * 1.5)
    a, e = inputs.encryption_randomness(77, 0, prm.q[:2], prm.n)
    ct = ckks.encrypt(prm, ev.sk, pt, a, e)
    a2, e2 = inputs.refresh_randomness(77, 0, prm.q, prm.n)
    fresh = ckks.refresh(prm, ev.sk, ct, a2, e2)
    assert fresh.level == prm.max_level and fresh.scale == ct.scale
    m_old = ckks.decrypt(prm, ev.sk, ct).m
    m_new = ckks.decrypt(prm, ev.sk, fresh).m
    # same plaintext polynomial plus the fresh encryption error, exactly
    want = ckks.add(m_old, ckks.reduce_signed(e2, prm.q[:2], prm.log_n), prm.q[:2])
    assert np.array_equal(m_new[:2], want)
    assert np.abs(ckks.decode(prm, ckks.decrypt(prm, ev.sk, fresh)) - z).max() < 1e-6
    # re-encoded at scale 2^40: the polynomial is round(m * 2^40 / scale), plus the fresh error
    re = ckks.refresh(prm, ev.sk, ct, a2, e2, prm.scale)
    assert re.scale == prm.scale and re.level == prm.max_level
    m0 = np.array([v - prm.q[0] if v > prm.q[0] // 2 else v for v in m_old[0].tolist()], dtype=np.int64)
    m1 = np.rint(m0 * (prm.scale / ct.scale)).astype(np.int64)
    want = ckks.add(ckks.reduce_signed(m1, prm.q[:2], prm.log_n), ckks.reduce_signed(e2, prm.q[:2], prm.log_n),
                    prm.q[:2])
    assert np.array_equal(ckks.decrypt(prm, ev.sk, re).m[:2], want)
    assert np.abs(ckks.decode(prm, ckks.decrypt(prm, ev.sk, re)) - z).max() < 1e-6


def test_encrypted_constant_operations():
    ev = make_oracle("toy", seed=78, relin=False, conj=False)
    prm = ev.prm
    z = inputs.slot_values(6, prm.slots)
    a, e = inputs.encryption_randomness(78, 0, prm.q[:3], prm.n)
    ct = ckks.encrypt(prm, ev.sk, ckks.encode(prm, z, 2, prm.scale), a, e)
    dec = lambda x: ckks.decode(prm, ckks.decrypt(prm, ev.sk, x))
    q2 = float(prm.q[2])
    assert np.abs(dec(ev.rescale(ev.cmult_const(ct, -0.3, q2))) + 0.3 * z).max() < 1e-7
    assert np.abs(dec(ev.cmult_const(ct, 7.0, 1.0)) - 7 * z).max() < 1e-7
    assert np.abs(dec(ev.add_const(ct, 2.5)) - (z + 2.5)).max() < 1e-7
    vals = inputs.slot_values(7, prm.slots)
    assert np.abs(dec(ev.add_plain(ct, vals)) - (z + vals)).max() < 1e-7


def refresher(ev, seed):
    count = [0]

    def refresh(ct):
        a, e = inputs.refresh_randomness(seed, count[0], ev.prm.q, ev.prm.n)
        count[0] += 1
        return ckks.refresh(ev.prm, ev.sk, ct, a, e, ev.prm.scale)
    return refresh


def test_encrypted_softmax_matches_the_simulator():
    """The encrypted algorithm (2^12 ring, 12 limbs, client refreshes) decrypts to the slot form."""
    s0, s1, c = 16, 128, 10
    ev = make_oracle("n12l12", seed=91, rot_steps=sm.rotation_steps(c, s1), conj=False)
    prm_c = ev.prm
    M = inputs.logits(70, 16, c, 32.0)
    cp = mx.next_pow2(c)
    blocks = tiled_blocks(M, cp, s0, s1)
    prm = sm.SoftmaxParams()
    cts = []
    for i, z in enumerate(blocks):
        a, e = inputs.encryption_randomness(91, i, prm_c.q[:9], prm_c.n)
        cts.append(ckks.encrypt(prm_c, ev.sk, ckks.encode(prm_c, z, 8, prm_c.scale), a, e))
    out, nref = sm.asoftmax_blocks(ev, cts, c, s0, s1, prm, sm.exp_coeffs(), prm_c.q, prm_c.max_level,
                                   refresher(ev, 91))
    sim = sm.ScaledSim(prm_c)
    sout, snref = sm.asoftmax_blocks(sim, [sim.encrypt(z, 8, prm_c.scale) for z in blocks], c, s0, s1, prm,
                                     sm.exp_coeffs(), prm_c.q, prm_c.max_level, sim.refresh)
    assert nref == snref
    for o, so in zip(out, sout):
        assert o.level == so.level and o.scale == pytest.approx(so.scale, rel=1e-12)
        got = ckks.decode(prm_c, ckks.decrypt(prm_c, ev.sk, o))
        assert np.abs(got - so.z).max() < 1e-4


def test_three_compositions_of_g_are_needed_at_ten_classes():
    """The reading Acomp = (f(g(g(g(.)))) + 1) / 2 against the text's f(g(g(.))) (App. softmax): with two
    compositions the maximum of 10 classes on [-128, 128] falls far enough below the true one that the sum
    of exponentials leaves AInv's range and Goldschmidt's iteration diverges, where Table softmaxerr prints
    finite errors for c = 10, R = 128; with three, the error is within that cell's printed maximum.
    The reading is a trade-off: at c = 3 the extra g costs accuracy (the sampled maximum error at R = 4 is
    about 3.5x that of two compositions), though it stays within 2x the printed maximum."""
    table = {(r["c"], r["R"]): r for r in json.load(open(os.path.join(GOLDEN, "softmax_err_table.json")))["rows"]}
    with np.errstate(all="ignore"):
        e2, _ = table_errors(10, 128, sm.SoftmaxParams(comp_g=2), 6000, 630)
    e3, _ = table_errors(10, 128, sm.SoftmaxParams(comp_g=3), 6000, 630)
    assert not np.isfinite(e2) or e2 > 1.0
    assert e3 <= table[(10, 128)]["prec"][0]
    c3_g2, _ = table_errors(3, 4, sm.SoftmaxParams(comp_g=2), 6000, 534)
    c3_g3, _ = table_errors(3, 4, sm.SoftmaxParams(comp_g=3), 6000, 534)
    assert c3_g2 < c3_g3 < 2.0 * table[(3, 4)]["prec"][0]
    assert c3_g3 > 2.5 * c3_g2
