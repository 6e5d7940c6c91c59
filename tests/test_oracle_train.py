"""Pins of the training-step oracle (Sec. 3's NAG update, the protocol's step 3(a))."""
import math

import numpy as np

from oracle import ckks
from oracle import matrix as mx
from oracle import softmax as sm
from oracle import train as tr
from paper_2403_14111_amd import inputs
from tests.oracle_setup import make_oracle
from tests.test_oracle_softmax import refresher


def test_nag_schedule():
    """lambda_{t+1}^2 - lambda_{t+1} = lambda_t^2 (the recursion solved), gamma_0 = 1, gamma_1 = 0, gamma_t -> -1."""
    assert tr.nag_gamma(0) == 1.0 and tr.nag_gamma(1) == 0.0
    lam = 0.0
    for t in range(50):
        nxt = (1.0 + math.sqrt(1.0 + 4.0 * lam * lam)) / 2.0
        assert abs(nxt * nxt - nxt - lam * lam) < 1e-9 * max(1.0, lam * lam)
        assert tr.nag_gamma(t) == (1.0 - lam) / nxt
        lam = nxt
    assert -1.0 < tr.nag_gamma(1000) < -0.99


def cross_entropy(X, Y, W):
    return -np.mean(np.sum(Y * np.log(sm.softmax_rows(X @ W.T)), axis=1))


def test_gradient_is_the_derivative_of_the_mean_cross_entropy():
    """(1/N)(P - Y)^T X against central differences, so the update's sign and transposes are the loss's."""
    rng = np.random.default_rng(3)
    X, W = rng.normal(size=(12, 7)), rng.normal(size=(4, 7)) * 0.3
    Y = np.eye(4)[rng.integers(0, 4, size=12)]
    g = (sm.softmax_rows(X @ W.T) - Y).T @ X / 12
    h = 1e-6
    num = np.zeros_like(W)
    for i in range(W.shape[0]):
        for j in range(W.shape[1]):
            E = np.zeros_like(W)
            E[i, j] = h
            num[i, j] = (cross_entropy(X, Y, W + E) - cross_entropy(X, Y, W - E)) / (2 * h)
    assert np.abs(g - num).max() < 1e-7
    Wn, Vn = tr.nag_step_plain(X, Y, W, W, 1.0, 1.0)
    assert np.allclose(Wn, W - 12 * g) and np.allclose(Vn, W)        # gamma = 1 keeps V at the old W


def test_nag_descends_on_a_separable_problem():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(40, 5))
    Y = np.eye(3)[np.argmax(X[:, :3], axis=1)]
    W = V = np.zeros((3, 5))
    losses = []
    for t in range(30):
        W, V = tr.nag_step_plain(X, Y, W, V, 0.5, tr.nag_gamma(t + 1))
        losses.append(cross_entropy(X, Y, W))
    assert losses[-1] < 0.5 * losses[0]


def encrypt_blocks(ev, mats, level, seed):
    out, idx = [], 0
    for row in mats:
        orow = []
        for z in row:
            a, e = inputs.encryption_randomness(seed, idx, ev.prm.q[:level + 1], ev.prm.n)
            orow.append(ckks.encrypt(ev.prm, ev.sk, ckks.encode(ev.prm, z, level, ev.prm.scale), a, e))
            idx += 1
        out.append(orow)
    return out


def train_case(seed=5):
    a, b, c = 20, 200, 10
    X = inputs.features(seed, a, b) * 0.25
    Y = np.eye(c)[inputs.labels(seed, a, c)]
    W = inputs.weights(seed, c, b, bound=0.2)
    V = inputs.weights(seed + 1, c, b, bound=0.2)
    return X, Y, W, V


def block_inputs(X, Y, W, V, c, s0, s1):
    cp = mx.next_pow2(c)
    pad = lambda M, r, cc: np.pad(M, ((0, r - M.shape[0]), (0, cc - M.shape[1])))
    xb = mx.block_encode(X, s0, s1)
    yb = [row[0] for row in mx.block_encode(mx.tile_horizontal(pad(Y, Y.shape[0], cp), s1), s0, s1)]
    wb = mx.block_encode(mx.tile_vertical(pad(W, cp, W.shape[1]), s0), s0, s1)[0]
    vb = mx.block_encode(mx.tile_vertical(pad(V, cp, V.shape[1]), s0), s0, s1)[0]
    return xb, yb, wb, vb


def test_encrypted_step_decrypts_to_the_plain_update():
    """The encrypted step (2^12 ring, 12 limbs, refreshes) against the FP64 update with the same ASoftmax."""
    s0, s1, c = 16, 128, 10
    X, Y, W, V = train_case()
    xb, yb, wb, vb = block_inputs(X, Y, W, V, c, s0, s1)
    steps = sorted(set(sm.rotation_steps(c, s1)) | set(mx.rotation_steps("abt", 16, s0, s1)) |
                   set(mx.rotation_steps("atb", 16, s0, s1)))
    ev = make_oracle("n12l12", seed=92, rot_steps=steps)
    X_ct = encrypt_blocks(ev, xb, 11, 93)
    Y_ct = encrypt_blocks(ev, [yb], 11, 94)[0]
    W_ct = encrypt_blocks(ev, [wb], 11, 95)[0]
    V_ct = encrypt_blocks(ev, [vb], 11, 96)[0]
    prm = sm.SoftmaxParams()
    lr, gamma = 0.5 / 20, tr.nag_gamma(3)
    Wn, Vn, nref = tr.nag_step_blocks(ev, X_ct, Y_ct, W_ct, V_ct, c, s0, s1, lr, gamma, prm, sm.exp_coeffs(),
                                      ev.prm.q, ev.prm.max_level, refresher(ev, 97))
    assert nref > 0
    dec = lambda cts: mx.block_decode([[ckks.decode(ev.prm, ckks.decrypt(ev.prm, ev.sk, x)).real for x in cts]],
                                      s0, s1)
    want_w, want_v = tr.nag_step_plain(X, Y, W, V, lr, gamma, lambda L: sm.asoftmax_rows(L, prm))
    got_w, got_v = dec(Wn), dec(Vn)
    assert np.abs(got_w[:c, :200] - want_w).max() < 1e-4
    assert np.abs(got_v[:c, :200] - want_v).max() < 1e-4
    for k in range(1, s0 // 16):                                  # the vertical tiling is kept
        assert np.abs(got_w[16 * k:16 * k + c, :200] - want_w).max() < 1e-4
    exact_w, _ = tr.nag_step_plain(X, Y, W, V, lr, gamma)
    assert np.abs(got_w[:c, :200] - exact_w).max() < 0.03 * lr * np.abs(X).sum(axis=0).max()
