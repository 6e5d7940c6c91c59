"""Oracle of the paper's encrypted matrix products (Sec. 4.2, App. B).

TEST INFRASTRUCTURE ONLY.  Written against an evaluator interface (rot, conj,
mult, cmult_mask, rescale, add, sub, mul_i, mod_drop, level) that both the
slot simulator (``slotsim.SimEvaluator``) and the encrypted oracle
(``ckks.Evaluator``) implement, so the operation counts pinned on the simulator
are the counts of the encrypted runs.

Block encoding (App. B.1): a matrix is zero padded to multiples of s0 x s1 and
cut into s0 x s1 blocks; block (i, j) is written row-major into one slot vector
of s = s0*s1 slots.

Readings taken where the paper is silent or inconsistent:
  * RU(B, k) on a block is Lrot(B, k*s1) (the row length of a block is s1).
  * CS: for m < log s1, x += Lrot(x, 2^m); multiply by the first-column mask
    and rescale; for m < log s1, x += Rrot(x, 2^m)  (2 log s1 rotations, one
    CMult, the count Sec. 4.2 states).
  * RS: for m < log s0, x += Lrot(x, 2^m s1)  (log s0 rotations, no depth).
  * DiagATB's mask is M^(-k, c) and its sum runs over k < c/2 (the proof of
    Prop. 2 and the complexification argument fix both).
  * Every product of a loop is taken at one common level, reached by dropping
    moduli, so that all terms rescale by the same prime; masks are encoded at
    scale q_level so that CMult + rescale keeps the scale.
  * A block product sum is relinearised per product and rescaled once.
"""
import numpy as np


# --------------------------------------------------------------------------
# Plain-matrix layout helpers (client side)
# --------------------------------------------------------------------------

def next_pow2(c):
    p = 1
    while p < c:
        p *= 2
    return p


def block_encode(mat, s0, s1):
    """Zero-pad and split into s0 x s1 blocks; returns slot vectors [n_rb][n_cb]."""
    mat = np.asarray(mat)
    rows, cols = mat.shape
    n_rb = -(-rows // s0)
    n_cb = -(-cols // s1)
    pad = np.zeros((n_rb * s0, n_cb * s1), dtype=mat.dtype)
    pad[:rows, :cols] = mat
    return [[pad[i * s0:(i + 1) * s0, j * s1:(j + 1) * s1].reshape(-1).copy() for j in range(n_cb)]
            for i in range(n_rb)]


def block_decode(blocks, s0, s1):
    """Inverse of block_encode (without removing padding)."""
    rows = [np.concatenate([np.asarray(b).reshape(s0, s1) for b in row], axis=1) for row in blocks]
    return np.concatenate(rows, axis=0)


def tile_vertical(b, s0):
    """B-bar: s0/c copies of the c x b matrix stacked vertically (s0 rows)."""
    c = b.shape[0]
    assert s0 % c == 0
    return np.tile(b, (s0 // c, 1))


def tile_horizontal(a, s1):
    """A-underbar: s1/c copies of the a x c matrix side by side (s1 columns)."""
    c = a.shape[1]
    assert s1 % c == 0
    return np.tile(a, (1, s1 // c))


# --------------------------------------------------------------------------
# Masks (slot vectors of one s0 x s1 block, row-major)
# --------------------------------------------------------------------------

def mask_offdiag(k, c, s0, s1):
    """M^(k, c): 1 where j == i + k (mod c)."""
    i = np.arange(s0)[:, None]
    j = np.arange(s1)[None, :]
    return (((j - i - k) % c) == 0).astype(np.float64).reshape(-1)


def mask_offdiag_cplx(k, c, s0, s1, t):
    """t * M_cplx^(k, c) = t/2 M^(k, c) - i t/2 M^(k + c/2, c)."""
    return t * (0.5 * mask_offdiag(k, c, s0, s1) - 0.5j * mask_offdiag(k + c // 2, c, s0, s1))


def mask_first_col(s0, s1):
    m = np.zeros((s0, s1))
    m[:, 0] = 1.0
    return m.reshape(-1)


def mask_left_cols(k, s0, s1):
    """D_k: 1 on columns j < s1 - k."""
    m = np.zeros((s0, s1))
    m[:, :s1 - k] = 1.0
    return m.reshape(-1)


def _log2(x):
    r = int(x).bit_length() - 1
    assert 1 << r == x, x
    return r


# --------------------------------------------------------------------------
# Block operations
# --------------------------------------------------------------------------

def col_sum(ev, x, s0, s1):
    """CS: every entry of a row becomes that row's sum."""
    lg = _log2(s1)
    for m in range(lg):
        x = ev.add(x, ev.rot(x, 1 << m))
    x = ev.rescale(ev.cmult_mask(x, mask_first_col(s0, s1)))
    for m in range(lg):
        x = ev.add(x, ev.rot(x, -(1 << m)))
    return x


def row_sum(ev, x, s0, s1):
    """RS: every entry of a column becomes that column's sum."""
    for m in range(_log2(s0)):
        x = ev.add(x, ev.rot(x, (1 << m) * s1))
    return x


def rot_left_cols(ev, a, k, s0, s1):
    """RL(A, k) (Alg. 2): columns rotated left by k inside each row; one level."""
    a1 = ev.rot(a, k)
    a2 = ev.rescale(ev.cmult_mask(a1, mask_left_cols(k, s0, s1)))
    rest = ev.sub(ev.mod_drop(a1, ev.level(a2)), a2)
    return ev.add(a2, ev.rot(rest, -s1))


def partial_rot_up(ev, b, k, s0, s1):
    """PRU(B, k) (Alg. 3): the last k columns move up by one row; one level."""
    bp = ev.rescale(ev.cmult_mask(b, mask_left_cols(k, s0, s1)))
    rest = ev.sub(ev.mod_drop(b, ev.level(bp)), bp)
    return ev.add(bp, ev.rot(rest, s1))


# --------------------------------------------------------------------------
# DiagABT (Alg. 1) and DiagATB (Alg. 4)
# --------------------------------------------------------------------------

def diag_abt(ev, A, Bbar, c, s0, s1, t=1.0):
    """<t A Bbar^T> from <A> (n_a x n_b blocks) and <Bbar> (1 x n_b blocks).

    Output: n_a blocks; block i slot (r, col) holds t (A B^T)[i s0 + r][col mod c].
    Requires 1 < c <= s0, c a power of two dividing s1.
    """
    assert 1 < c <= s0 and s1 % c == 0 and c & (c - 1) == 0
    n_a, n_b = len(A), len(A[0])
    assert len(Bbar) == n_b
    lv = min(min(ev.level(x) for row in A for x in row), min(ev.level(x) for x in Bbar))
    A = [[ev.mod_drop(x, lv) for x in row] for row in A]
    Bbar = [ev.mod_drop(x, lv) for x in Bbar]
    half = c // 2
    b_cplx = [ev.add(b, ev.mul_i(ev.rot(b, half * s1))) for b in Bbar]
    X = [None] * n_a
    for k in range(half):
        b_k = b_cplx if k == 0 else [ev.rot(b, k * s1) for b in b_cplx]
        mask = mask_offdiag_cplx(k, c, s0, s1, t)
        for i in range(n_a):
            r = None
            for j in range(n_b):
                p = ev.mult(A[i][j], b_k[j])
                r = p if r is None else ev.add(r, p)
            r = ev.rescale(r)
            r = col_sum(ev, r, s0, s1)
            r = ev.rescale(ev.cmult_mask(r, mask))
            X[i] = r if X[i] is None else ev.add(X[i], r)
    return [ev.add(x, ev.conj(x)) for x in X]


def diag_atb(ev, Abar, B, c, s0, s1, t=1.0):
    """<t Abar^T B> from <Abar> (n_a x 1 blocks, A tiled horizontally) and <B> (n_a x n_b).

    Output: n_b blocks; block j slot (r, col) holds t (A^T B)[r mod c][j s1 + col].
    The PRotUp branch is taken when level(Abar) < level(B).
    """
    assert 1 < c <= s1 and s1 % c == 0 and c & (c - 1) == 0
    n_a = len(Abar)
    n_b = len(B[0])
    assert len(B) == n_a and all(len(a) == 1 for a in Abar)
    Abar = [a[0] for a in Abar]
    lA = min(ev.level(x) for x in Abar)
    lB = min(ev.level(x) for row in B for x in row)
    Abar = [ev.mod_drop(x, lA) for x in Abar]
    B = [[ev.mod_drop(x, lB) for x in row] for row in B]
    use_pru = lA < lB
    half = c // 2
    a_cplx = []
    for a in Abar:
        rl = rot_left_cols(ev, a, half, s0, s1)
        a_cplx.append(ev.add(ev.mod_drop(a, ev.level(rl)), ev.mul_i(rl)))
    lvl_star = min(lA - 1, lB - 1) if use_pru else min(lA - 2, lB)
    X = [None] * n_b
    for k in range(half):
        if use_pru:
            a_k = [ev.mod_drop(a if k == 0 else ev.rot(a, k), lvl_star) for a in a_cplx]
            b_k = [[ev.mod_drop(b if k == 0 else partial_rot_up(ev, b, k, s0, s1), lvl_star) for b in row]
                   for row in B]
        else:
            a_k = [ev.mod_drop(a if k == 0 else rot_left_cols(ev, a, k, s0, s1), lvl_star) for a in a_cplx]
            b_k = [[ev.mod_drop(b, lvl_star) for b in row] for row in B]
        mask = mask_offdiag_cplx(-k, c, s0, s1, t)
        for j in range(n_b):
            r = None
            for i in range(n_a):
                p = ev.mult(a_k[i], b_k[i][j])
                r = p if r is None else ev.add(r, p)
            r = ev.rescale(r)
            r = row_sum(ev, r, s0, s1)
            r = ev.rescale(ev.cmult_mask(r, mask))
            X[j] = r if X[j] is None else ev.add(X[j], r)
    return [ev.add(x, ev.conj(x)) for x in X]


def rotation_steps(op, c, s0, s1, n_a=1, n_b=1, pru=False):
    """Left-rotation amounts (negative: right) the algorithms call, for key generation."""
    steps = set()
    half = c // 2
    if op == "abt":
        steps.update(k * s1 for k in range(1, half + 1))
        steps.update(1 << m for m in range(_log2(s1)))
        steps.update(-(1 << m) for m in range(_log2(s1)))
    elif op == "atb":
        steps.update(range(1, half + 1))
        steps.add(-s1)
        steps.update((1 << m) * s1 for m in range(_log2(s0)))
        if pru:
            steps.add(s1)
    else:
        raise ValueError(op)
    return sorted(steps)
