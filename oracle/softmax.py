"""Oracle of the paper's row-wise softmax approximation (App. "Softmax approximation":
Alg. "Row-wise softmax approximation", Thm. "softmaxbound", the parameter list of the
comparison subsection and Table "softmaxerr").

TEST INFRASTRUCTURE ONLY.  Two forms of the same algorithm:
  * ``asoftmax_rows``: plain FP64 on row vectors (many at once), for the error analysis;
  * ``asoftmax_blocks``: the encrypted algorithm on block-encoded, horizontally tiled
    matrices, written against an evaluator interface that the slot simulator
    (``ScaledSim``) and the encrypted oracle (``ckks.Evaluator``) both implement.

What the algorithm computes (App. softmax): ASoftmax = p o D_n o Norm, where Norm subtracts an
approximate row maximum Amax (pairwise, Amax(a, b) = a Acomp(a, b) + b (1 - Acomp(a, b)) with
Acomp(a, b) ~ (sgn(a - b) + 1) / 2 = (f(g(..g(a - b))) + 1) / 2 on [-1/2, 1/2]), D_n is the domain
extension polynomial of n steps d_i(x) = L^i B(x / L^i), B(x) = x - 4 x^3 / (27 R^2), applied for
i = n-1 .. 0 (optionally followed by the degree-5 correction B_inv), and p is softmax on [-R, R]
evaluated as AExp(x) / sum AExp with AInv for the reciprocal.

Readings (the paper is silent or garbled here; each is also listed with the design notes):
  * R = 8 (AExp's range), L = 2, n = 5: the inputs may lie in [-128, 128]; R_max = ceil(R L^n).
  * M_max starts as M' (it is used before being set); the max loop runs log2 c' times.
  * Acomp = (f(g(g(g(a - b)))) + 1) / 2, three compositions of g: with the listing's input scale
    1 / (2 R_max), f(g(g(.))) leaves the maximum of 10 classes up to ~6 below the true one on
    [-8, 8], the sum of exponentials then exceeds AInv's range (2 R_inv) and the iteration
    diverges, where Table softmaxerr reports finite errors; one more g reproduces the table.
  * B_inv(x) = x + k (x^3 / R^2 - x^5 / R^4): the approximate inverse of D_n near 0 (the printed
    sign makes the error grow, against the table's "+prec" column).
  * The max is broadcast along the row by Rrot(x, 2^j), j < log2 s1 (the printed 2^i s1 would
    move it across rows).
  * "x (2 R_max)" multiplies by the integer 2 R_max (exact, no level); "x 1/(2 R_max)" and every
    other real constant is encoded at scale q_level and rescaled, which keeps the scale.
  * D_c is 1 on the first c columns of each row (the first period of the tiling): the last lines
    rebuild the tiling from that period.
  * AExp(x) = p(x / B)^B with B = 8, p the degree-12 least-squares (L^2) approximation of e^t
    on [-1, 1] (the cited method with the paper's B = 8); x / B is folded into p's coefficients.
  * The row sum ("RS" in the listing) runs over the c' columns of the first period, CS-style:
    x += Lrot(x, 2^j) for j < log2 c', the first-column mask, x += Rrot(x, 2^j) for j < log2 c'.
  * AInv(x) = Goldschmidt's iteration on y = x / R_inv, R_inv = 100, 16 steps: a = 2 - y,
    b = 1 - y, then b <- b^2, a <- a (1 + b); 1/x ~ a / R_inv.  Before it the slots outside the
    first period are set to 1 (plaintext add), keeping them in AInv's domain (0, R_inv].
  * M_sm = M_exp (x) M_Z (the listing multiplies the sum by its own inverse), then replicated by
    Rrot(x, 2^j c'), j < log2(s1 / c') (the printed stride 2^j s1 c' leaves the row).
  * Polynomials are evaluated in the power basis: x^k = x^a x^b with a the largest power of two
    below k (a = b = k/2 for k a power of two), each product relinearised and rescaled; every
    term c_k x^k is brought to the common level by mod-drop and multiplied by c_k encoded at the
    scale that lands on the input's scale; the constant term is added last.
  * Levels: an operand whose level is below what the next step needs is refreshed (handed back
    to the key holder and re-encrypted at the top level and the scale 2^40, see ``ckks.refresh``);
    the paper bootstraps instead.  Re-encoding at a fixed scale matters: Goldschmidt's 16
    squarings double the scale's log distance from the primes at every step, which at N = 2^16
    (primes up to 5e-6 below 2^40) would leave the output at scale ~2^52 and overflow the
    constants of a following training step.  Sums of ciphertexts whose scales differ bring the second operand to
    the first's scale with a constant 1 encoded at the matching scale (one level).

Parity status: pinned.  The plain form is pinned by the closed form of f, the DEP lemmas, the
theorem's bound and Table softmaxerr (tests/test_oracle_softmax.py).  The coefficients of p and
the AInv parameters are not printed in the paper: p is pinned to its closed form (the truncated
Legendre series of e^t, coefficients (2n + 1) i_n(1) from the modified spherical Bessel functions)
and AInv to the closed form of Goldschmidt's iteration, (1 - (1 - x / R)^(2^17)) / x; the
parameter choices themselves (degree 12, B = 8, R = 100, 16 steps) are readings, checked only
through Table softmaxerr.
"""
import math

import numpy as np

from . import ckks

# f and g of the comparison (App. softmax), as integer numerators over a power-of-two denominator.
F_NUM, F_DEN = (0, 35, 0, -35, 0, 21, 0, -5), 16
G_NUM, G_DEN = (0, 4589, 0, -16577, 0, 25614, 0, -12860), 1024


class SoftmaxParams:
    def __init__(self, R=8.0, L=2.0, n=5, precise=True, exp_B=8, exp_degree=12, inv_R=100.0, inv_iters=16,
                 comp_g=3, extend=True):
        self.R, self.L, self.n, self.precise = float(R), float(L), int(n), bool(precise)
        self.exp_B, self.exp_degree = int(exp_B), int(exp_degree)
        self.inv_R, self.inv_iters, self.comp_g = float(inv_R), int(inv_iters), int(comp_g)
        self.extend = bool(extend)
        if self.exp_B & (self.exp_B - 1):
            raise ValueError("exp_B must be a power of two")

    @property
    def r_max(self):
        return math.ceil(self.R * self.L ** (self.n if self.extend else 0))


def f_coeffs():
    return [v / F_DEN for v in F_NUM]


def g_coeffs():
    return [v / G_DEN for v in G_NUM]


def comp_out_coeffs():
    """(f + 1) / 2: the last polynomial of Acomp."""
    c = [v / (2 * F_DEN) for v in F_NUM]
    c[0] = 0.5
    return c


def dep_coeffs(prm, i):
    """d_i(x) = L^i B(x / L^i) = x - 4 x^3 / (27 R^2 L^(2i))."""
    return [0.0, 1.0, 0.0, -4.0 / (27.0 * prm.R * prm.R * prm.L ** (2 * i))]


def dep_inv_coeffs(prm):
    """B_inv(x) = x + k (x^3 / R^2 - x^5 / R^4), k = 4 L^2 (L^(2n) - 1) / (27 L^(2n) (L^2 - 1)): near 0,
    D_n(x) = x - k x^3 / R^2 + O(x^5), and this is its approximate inverse (reading: the printed
    sign of the bracket would double the distortion instead of undoing it)."""
    l2, l2n = prm.L ** 2, prm.L ** (2 * prm.n)
    k = 4.0 * l2 * (l2n - 1.0) / (27.0 * l2n * (l2 - 1.0))
    return [0.0, 1.0, 0.0, k / (prm.R ** 2), 0.0, -k / (prm.R ** 4)]


def exp_coeffs(degree=12, B=8):
    """Monomial coefficients of p(x / B), p the L^2-projection of e^t onto polynomials of degree
    <= `degree` on [-1, 1] (Legendre coefficients by Gauss-Legendre quadrature, exact for this
    degree up to rounding)."""
    x, w = np.polynomial.legendre.leggauss(64)
    ex = np.exp(x)
    leg = np.empty(degree + 1)
    for k in range(degree + 1):
        pk = np.polynomial.legendre.Legendre.basis(k)(x)
        leg[k] = (2 * k + 1) / 2.0 * np.sum(w * ex * pk)
    mono = np.polynomial.legendre.leg2poly(leg)
    return [float(mono[k]) / float(B) ** k for k in range(degree + 1)]


# --------------------------------------------------------------------------
# Plain FP64 form on row vectors
# --------------------------------------------------------------------------

def _pv(coeffs, x):
    return np.polynomial.polynomial.polyval(x, np.asarray(coeffs, dtype=np.float64))


def acomp_plain(a, b, prm):
    y = a - b
    for _ in range(prm.comp_g):
        y = _pv(g_coeffs(), y)
    return _pv(comp_out_coeffs(), y)


def amax_plain(xs, prm):
    """Row maxima by the pairwise tree of the listing: after round j, entry i holds Amax over the
    cyclic window [i, i + 2^(j+1)) of the c'-periodic row; entry 0 is returned."""
    m = np.array(xs, dtype=np.float64)
    cp = m.shape[1]
    j = 1
    while j < cp:
        rot = np.roll(m, -j, axis=1)
        comp = acomp_plain(m, rot, prm)
        m = m * comp + rot * (1.0 - comp)
        j *= 2
    return m[:, 0]


def dep_plain(x, prm):
    for i in range(prm.n - 1, -1, -1):
        x = _pv(dep_coeffs(prm, i), x)
    if prm.precise:
        x = _pv(dep_inv_coeffs(prm), x)
    return x


def aexp_plain(x, prm, coeffs=None):
    coeffs = exp_coeffs(prm.exp_degree, prm.exp_B) if coeffs is None else coeffs
    y = _pv(coeffs, x)
    b = prm.exp_B
    while b > 1:
        y = y * y
        b //= 2
    return y


def ainv_plain(x, prm):
    y = x / prm.inv_R
    b = 1.0 - y
    a = 2.0 - y
    for _ in range(prm.inv_iters):
        b = b * b
        a = a * (1.0 + b)
    return a / prm.inv_R


def asoftmax_rows(X, prm, exp_c=None):
    """ASoftmax of each row of X (k x c), plain FP64, in the listing's order."""
    X = np.asarray(X, dtype=np.float64)
    k, c = X.shape
    cp = 1
    while cp < c:
        cp *= 2
    xs = np.full((k, cp), -0.5)
    xs[:, :c] = X / (2.0 * prm.r_max)
    m = amax_plain(xs, prm) * (2.0 * prm.r_max)
    xn = X - m[:, None]
    if prm.extend:
        xn = dep_plain(xn, prm)
    e = aexp_plain(xn, prm, exp_c)
    s = e.sum(axis=1)
    z = ainv_plain(s, prm)
    return e * z[:, None]


def softmax_rows(X):
    X = np.asarray(X, dtype=np.float64)
    e = np.exp(X - X.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def beta_bound(c, delta, r, L):
    """The theorem's bound beta(c, delta, r, L, d) on |Softmax - p o D_n o Norm| - eps."""
    t = delta * L * L * r ** 3 / (L * L - 1.0)
    return 1.0 / (1.0 + math.exp(r) / (c - 1)) + 1.0 / (1.0 + math.exp(r - t) / (c - 1)) + t / 2.0


# --------------------------------------------------------------------------
# Block-encoded form over an evaluator
# --------------------------------------------------------------------------

def _split(k):
    a = 1 << (k.bit_length() - 1)
    return (k // 2, k // 2) if a == k else (a, k - a)


def power_depth(k):
    if k <= 1:
        return 0
    a, b = _split(k)
    return max(power_depth(a), power_depth(b)) + 1


def poly_depth(coeffs):
    ks = [k for k in range(1, len(coeffs)) if coeffs[k] != 0.0]
    return max(power_depth(k) for k in ks) + 1 if ks else 0


def _needed_powers(coeffs):
    need = set()
    stack = [k for k in range(1, len(coeffs)) if coeffs[k] != 0.0]
    while stack:
        k = stack.pop()
        if k in need:
            continue
        need.add(k)
        if k > 1:
            stack.extend(_split(k))
    return sorted(need)


class Steps:
    """The algorithm's building blocks over an evaluator `ev` on lists of ciphertexts (one per row
    block, all at one level and scale), with the level rule: an operand below the depth a step
    needs is first passed to `refresh` (each block in order)."""

    def __init__(self, ev, q, max_level, refresh=None):
        self.ev, self.q, self.max_level, self.refresh_fn = ev, q, max_level, refresh
        self.refreshes = 0

    def level(self, xs):
        return self.ev.level(xs[0])

    def need(self, xs, d):
        if self.level(xs) >= d:
            return xs
        if self.refresh_fn is None or d > self.max_level:
            raise ckks.LevelError("depth budget exhausted (needs %d levels, has %d)" % (d, self.level(xs)))
        out = []
        for x in xs:
            out.append(self.refresh_fn(x))
            self.refreshes += 1
        return out

    def drop(self, xs, lv):
        return xs if self.level(xs) == lv else [self.ev.mod_drop(x, lv) for x in xs]

    def rescale(self, xs):
        return [self.ev.rescale(x) for x in xs]

    def cconst(self, xs, v):
        """x * v with v encoded at scale q_level, rescaled (scale kept, one level)."""
        xs = self.need(xs, 1)
        q = float(self.q[self.level(xs)])
        return self.rescale([self.ev.cmult_const(x, v, q) for x in xs])

    def mulint(self, xs, k):
        return [self.ev.cmult_const(x, float(k), 1.0) for x in xs]

    def add_const(self, xs, v):
        return [self.ev.add_const(x, v) for x in xs]

    def add_plain(self, xs, values):
        return [self.ev.add_plain(x, values) for x in xs]

    def mask(self, xs, values):
        xs = self.need(xs, 1)
        return self.rescale([self.ev.cmult_mask(x, values) for x in xs])

    def rot(self, xs, r):
        return [self.ev.rot(x, r) for x in xs]

    def mult(self, a, b):
        same = a is b
        a = self.need(a, 1)
        b = a if same else self.need(b, 1)
        lv = min(self.level(a), self.level(b))
        a, b = self.drop(a, lv), self.drop(b, lv)
        return self.rescale([self.ev.mult(x, y) for x, y in zip(a, b)])

    def _combine(self, a, b, subtract):
        sa, sb = a[0].scale, b[0].scale
        if abs(sa - sb) > 1e-9 * max(abs(sa), abs(sb)):
            b = self.need(b, 1)
            q = float(self.q[self.level(b)])
            sigma = sa * q / sb
            b = self.rescale([self.ev.cmult_const(x, 1.0, sigma) for x in b])
        lv = min(self.level(a), self.level(b))
        a, b = self.drop(a, lv), self.drop(b, lv)
        op = self.ev.sub if subtract else self.ev.add
        return [op(x, y) for x, y in zip(a, b)]

    def add(self, a, b):
        return self._combine(a, b, False)

    def sub(self, a, b):
        return self._combine(a, b, True)

    def poly(self, xs, coeffs):
        """sum_k coeffs[k] x^k in the power basis (see the module notes); the result has the
        input's scale (to rounding) and sits poly_depth(coeffs) levels below the input."""
        ks = [k for k in range(1, len(coeffs)) if coeffs[k] != 0.0]
        if not ks:
            raise ValueError("constant polynomial")
        xs = self.need(xs, poly_depth(coeffs))
        target = xs[0].scale
        pw = {1: xs}
        for k in _needed_powers(coeffs):
            if k > 1:
                a, b = _split(k)
                pw[k] = self.mult(pw[a], pw[b])
        lt = min(self.level(pw[k]) for k in ks) - 1
        q = float(self.q[lt + 1])
        acc = None
        for k in ks:
            t = self.drop(pw[k], lt + 1)
            sigma = target * q / t[0].scale
            t = self.rescale([self.ev.cmult_const(x, coeffs[k], sigma) for x in t])
            acc = t if acc is None else [self.ev.add(u, v) for u, v in zip(acc, t)]
        if coeffs[0] != 0.0:
            acc = self.add_const(acc, coeffs[0])
        return acc


def _cols(s0, s1, pred, value):
    j = np.arange(s1)
    row = np.where(pred(j), value, 0.0)
    return np.tile(row, s0).astype(np.complex128)


def asoftmax_blocks(ev, xs, c, s0, s1, prm, exp_c, q, max_level, refresh=None):
    """Alg. softmax on the row blocks `xs` of a horizontally tiled a x c matrix (each row of a block
    holds the c' padded classes repeated s1 / c' times).  Returns (blocks, number of refreshes)."""
    cp = 1
    while cp < c:
        cp *= 2
    if cp > s1 or s1 % cp:
        raise ValueError("c' must divide s1")
    S = Steps(ev, q, max_level, refresh)
    d_c = _cols(s0, s1, lambda j: j < c, 1.0)
    first = _cols(s0, s1, lambda j: j == 0, 1.0)
    rmax = prm.r_max

    x0 = S.need(list(xs), 1)
    x = S.cconst(x0, 1.0 / (2.0 * rmax))
    if c != cp:
        x = S.add_plain(x, _cols(s0, s1, lambda j: j % cp >= c, -0.5))
    # normalisation: approximate row maximum (pairwise comparisons), broadcast along the row
    mmax = x
    j = 1
    while j < cp:
        mrot = S.rot(mmax, j)
        y = S.sub(mmax, mrot)
        for _ in range(prm.comp_g):
            y = S.poly(y, g_coeffs())
        comp = S.poly(y, comp_out_coeffs())
        onem = S.add_const(S.mulint(comp, -1), 1.0)
        mmax = S.add(S.mult(mmax, comp), S.mult(mrot, onem))
        j *= 2
    mmax = S.mask(mmax, first)
    j = 1
    while j < s1:
        mmax = S.add(mmax, S.rot(mmax, -j))
        j *= 2
    mmax = S.mulint(mmax, 2 * rmax)
    xn = S.mask(S.sub(x0, mmax), d_c)
    # domain extension
    if prm.extend:
        for i in range(prm.n - 1, -1, -1):
            xn = S.poly(xn, dep_coeffs(prm, i))
        if prm.precise:
            xn = S.poly(xn, dep_inv_coeffs(prm))
    # exponential, row sum over the first period, reciprocal
    e = S.poly(xn, exp_c)
    b = prm.exp_B
    while b > 1:
        e = S.mult(e, e)
        b //= 2
    e = S.mask(e, d_c)
    s = e
    j = 1
    while j < cp:
        s = S.add(s, S.rot(s, j))
        j *= 2
    s = S.mask(s, first)
    j = 1
    while j < cp:
        s = S.add(s, S.rot(s, -j))
        j *= 2
    s = S.add_plain(s, _cols(s0, s1, lambda jj: jj >= cp, 1.0))
    y = S.cconst(s, 1.0 / prm.inv_R)
    bq = S.add_const(S.mulint(y, -1), 1.0)
    a = S.add_const(bq, 1.0)
    for _ in range(prm.inv_iters):
        bq = S.mult(bq, bq)
        a = S.mult(a, S.add_const(bq, 1.0))
    z = S.cconst(a, 1.0 / prm.inv_R)
    sm = S.mult(e, z)
    j = cp
    while j < s1:
        sm = S.add(sm, S.rot(sm, -j))
        j *= 2
    return sm, S.refreshes


def rotation_steps(c, s1):
    """Rotation amounts the algorithm uses."""
    cp = 1
    while cp < c:
        cp *= 2
    steps = set()
    j = 1
    while j < cp:
        steps |= {j, -j}
        j *= 2
    j = 1
    while j < s1:
        steps.add(-j)
        j *= 2
    j = cp
    while j < s1:
        steps.add(-j)
        j *= 2
    return sorted(steps)


# --------------------------------------------------------------------------
# Slot simulator with the encrypted evaluator's level and scale bookkeeping
# --------------------------------------------------------------------------

class ScaledSim:
    """Slot vectors with the exact level and FP64 scale bookkeeping of ``ckks.Evaluator`` (the
    primes of a parameter set), so that refresh points and scale alignments match the encrypted
    run; values are exact FP64 (no encoding rounding, no noise)."""

    class Ct:
        def __init__(self, z, level, scale):
            self.z, self.level, self.scale = np.asarray(z, dtype=np.complex128), int(level), float(scale)

    def __init__(self, prm):
        self.prm = prm
        self.counts = {}

    def _count(self, name):
        self.counts[name] = self.counts.get(name, 0) + 1

    @staticmethod
    def level(x):
        return x.level

    def encrypt(self, z, level, scale):
        return ScaledSim.Ct(z, level, scale)

    def _pair(self, a, b):
        if a.level != b.level or abs(a.scale - b.scale) > 1e-9 * max(a.scale, b.scale):
            raise ValueError("level or scale mismatch")

    def add(self, a, b):
        self._pair(a, b)
        return ScaledSim.Ct(a.z + b.z, a.level, a.scale)

    def sub(self, a, b):
        self._pair(a, b)
        return ScaledSim.Ct(a.z - b.z, a.level, a.scale)

    def mod_drop(self, a, lv):
        if lv > a.level or lv < 0:
            raise ckks.LevelError("bad mod drop")
        return ScaledSim.Ct(a.z, lv, a.scale)

    def rescale(self, a):
        if a.level < 1:
            raise ckks.LevelError("no level left to rescale")
        return ScaledSim.Ct(a.z, a.level - 1, a.scale / self.prm.q[a.level])

    def cmult_const(self, a, v, sigma):
        self._count("cmult_const")
        return ScaledSim.Ct(a.z * v, a.level, a.scale * float(sigma))

    def add_const(self, a, v):
        return ScaledSim.Ct(a.z + v, a.level, a.scale)

    def add_plain(self, a, values):
        return ScaledSim.Ct(a.z + values, a.level, a.scale)

    def cmult_mask(self, a, values):
        self._count("cmult")
        return ScaledSim.Ct(a.z * values, a.level, a.scale * float(self.prm.q[a.level]))

    def mult(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")
        self._count("mult")
        return ScaledSim.Ct(a.z * b.z, a.level, a.scale * b.scale)

    def rot(self, a, r):
        self._count("rot")
        return ScaledSim.Ct(np.roll(a.z, -r), a.level, a.scale)

    def refresh(self, a):
        """The key holder's refresh: top level, re-encoded at the parameter set's scale."""
        return ScaledSim.Ct(a.z, self.prm.max_level, self.prm.scale)
