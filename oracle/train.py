"""Oracle of one step of the encrypted training loop (the protocol's step 3(a) and Sec. 3's NAG update):

    P       = ASoftmax(X V_t^T)
    W_{t+1} = V_t - (alpha / N) (P - Y)^T X
    V_{t+1} = (1 - gamma_t) W_{t+1} + gamma_t W_t,   gamma_t = (1 - lambda_t) / lambda_{t+1},
    lambda_0 = 0, lambda_{t+1} = (1 + sqrt(1 + 4 lambda_t^2)) / 2.

TEST INFRASTRUCTURE ONLY.  ``nag_step_plain`` is the FP64 update (with any softmax); ``nag_step_blocks``
is the encrypted step over an evaluator: X untiled (n_a x n_b blocks), Y one-hot and tiled horizontally
(n_a blocks), W and V tiled vertically (n_b blocks); the logits come from DiagABT (Alg. 1), the gradient from
DiagATB (Alg. 4) with t = -alpha / N.  Levels follow the softmax oracle's rule: X and V are refreshed below 3
levels (DiagABT's depth), P - Y below 4 (DiagATB's RotLeft branch), and sums align scales as there.

Parity status: pinned against the plain update (tests/test_oracle_train.py).
"""
import math

import numpy as np

from . import matrix as mx
from . import softmax as sm


def nag_gamma(t):
    """gamma_t of the NAG schedule (Sec. 3)."""
    lam = 0.0
    for _ in range(t):
        lam = (1.0 + math.sqrt(1.0 + 4.0 * lam * lam)) / 2.0
    nxt = (1.0 + math.sqrt(1.0 + 4.0 * lam * lam)) / 2.0
    return (1.0 - lam) / nxt


def nag_step_plain(X, Y, W, V, lr, gamma, softmax=sm.softmax_rows):
    """FP64: (W_{t+1}, V_{t+1}); lr = alpha / N."""
    P = softmax(X @ V.T)
    Wn = V - lr * (P - Y).T @ X
    return Wn, (1.0 - gamma) * Wn + gamma * W


def nag_step_blocks(ev, X, Y, W, V, c, s0, s1, lr, gamma, prm, exp_c, q, max_level, refresh=None):
    """The encrypted step: X [[ct]] (n_a x n_b), Y [ct] (n_a), W and V [ct] (n_b).  Returns (W_{t+1}, V_{t+1},
    number of refreshes)."""
    cp = mx.next_pow2(c)
    S = sm.Steps(ev, q, max_level, refresh)
    n_b = len(X[0])
    flat = S.need([x for row in X for x in row], 3)
    Xr = [flat[i * n_b:(i + 1) * n_b] for i in range(len(X))]
    Vr = S.need(list(V), 3)
    logits = mx.diag_abt(ev, Xr, Vr, cp, s0, s1, 1.0)
    P, nref = sm.asoftmax_blocks(ev, logits, c, s0, s1, prm, exp_c, q, max_level, refresh)
    D = S.need(S.sub(P, list(Y)), 4)
    G = mx.diag_atb(ev, [[d] for d in D], Xr, cp, s0, s1, -lr)
    Wn = S.add(Vr, G)
    a = S.cconst(Wn, 1.0 - gamma)
    b = S.cconst(list(W), gamma)
    Vn = S.add(a, b)
    return Wn, Vn, S.refreshes + nref
