"""GPU parity of one encrypted training step (NAG, Sec. 3): logits by DiagABT, ASoftmax, P - Y, the gradient by
DiagATB, the NAG combination; refreshes included, word for word against the oracle."""
import sys

import numpy as np
import pytest

from oracle import matrix as mx
from oracle import softmax as sm
from oracle import train as tr
from paper_2403_14111_amd import inputs
from tests.golden_data import aexp_coeffs
from tests.gpu_setup import make_gpu, softmax_params_with
from tests.oracle_setup import make_oracle
from tests.test_gpu_parity import compare_blocks, enc_mat_both
from tests.test_oracle_softmax import refresher as oracle_refresher
from tests.test_oracle_train import train_case

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] train " + msg, file=sys.stderr, flush=True)


def test_nag_step_bit_exact():
    s0, s1, c = 16, 128, 10
    cp = mx.next_pow2(c)
    steps = sorted(set(sm.rotation_steps(c, s1)) | set(mx.rotation_steps("abt", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1, pru=True)))
    note("n12l12 context + keys (%d rotations)" % len(steps))
    ctx, sk, keys = make_gpu("n12l12", seed=2500, rot_steps=steps)
    ev = make_oracle("n12l12", seed=2500, rot_steps=steps)
    X, Y, W, V = train_case()
    gx, ox = enc_mat_both(ctx, sk, ev, X, s0, 11, 0, cp, seed=101)
    gy, oy = enc_mat_both(ctx, sk, ev, Y, s0, 11, 2, cp, seed=102)
    gw, ow = enc_mat_both(ctx, sk, ev, W, s0, 11, 1, cp, seed=103)
    gv, ov = enc_mat_both(ctx, sk, ev, V, s0, 11, 1, cp, seed=104)
    lr, gamma = 0.5 / 20, tr.nag_gamma(3)
    note("gpu step")
    gr = ctx.refresher(sk, lambda i: inputs.refresh_randomness(2501, i, ctx.q, ctx.n))
    exp_c = aexp_coeffs()
    gW, gV, nref = ctx.nag_step(keys, gx, gy, gw, gv, c, lr, gamma, params=softmax_params_with(exp_c), refresh=gr)
    note("oracle step")
    prm = sm.SoftmaxParams()
    oW, oV, onref = tr.nag_step_blocks(ev, ox, [r[0] for r in oy], ow[0], ov[0], c, s0, s1, lr, gamma, prm,
                                       exp_c, ev.prm.q, ev.prm.max_level, oracle_refresher(ev, 2501))
    assert nref == onref == gr.calls[0]
    assert (gW.level, gV.level) == (oW[0].level, oV[0].level)
    compare_blocks(ctx, gW, oW)
    compare_blocks(ctx, gV, oV)
    want_w, want_v = tr.nag_step_plain(X, Y, W, V, lr, gamma, lambda L: sm.asoftmax_rows(L, prm))
    assert np.abs(ctx.mat_decrypt(sk, gW)[:c, :200] - want_w).max() < 1e-4
    assert np.abs(ctx.mat_decrypt(sk, gV)[:c, :200] - want_v).max() < 1e-4


def test_nag_step_full_ring():
    """N = 2^16, the benchmark's 128 x 769 x 10 step (features with a bias column), against the plain update."""
    s0, c, cp = 128, 10, 16
    s1 = 32768 // s0
    steps = sorted(set(sm.rotation_steps(c, s1)) | set(mx.rotation_steps("abt", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1, pru=True)))
    note("full ring context + keys (%d rotations)" % len(steps))
    ctx, sk, keys = make_gpu("n16l12", seed=2600, rot_steps=steps)
    X = np.hstack([inputs.features(1002, 128, 768), np.ones((128, 1))])
    Y = np.eye(c)[inputs.labels(1002, 128, c)]
    W = inputs.weights(1002, c, 769)
    V = inputs.weights(1003, c, 769)

    def enc(M, tiling, seed):
        nb = int(np.prod(ctx.mat_blocks(M.shape[0], M.shape[1], s0, tiling, cp)))
        r = [inputs.encryption_randomness(seed, b, ctx.q[:12], ctx.n) for b in range(nb)]
        return ctx.mat_encrypt(sk, M, s0, 11, 2.0 ** 40, np.stack([x[0] for x in r]), np.stack([x[1] for x in r]),
                               tiling=tiling, c=cp)
    gx, gy, gw, gv = enc(X, 0, 201), enc(Y, 2, 202), enc(W, 1, 203), enc(V, 1, 204)
    lr, gamma = 1.0 / 128, tr.nag_gamma(2)
    note("full ring step")
    gr = ctx.refresher(sk, lambda i: inputs.refresh_randomness(2601, i, ctx.q, ctx.n))
    gW, gV, nref = ctx.nag_step(keys, gx, gy, gw, gv, c, lr, gamma, refresh=gr)
    assert nref > 0
    prm = sm.SoftmaxParams()
    want_w, want_v = tr.nag_step_plain(X, Y, W, V, lr, gamma, lambda L: sm.asoftmax_rows(L, prm))
    assert np.abs(ctx.mat_decrypt(sk, gW)[:c, :769] - want_w).max() < 1e-4
    assert np.abs(ctx.mat_decrypt(sk, gV)[:c, :769] - want_v).max() < 1e-4


def test_nag_step_config3_full_ring():
    """N = 2^16, the survey's config 3: 256 x 769 features (with the bias column), 100 classes -> c' = 128, s0 = 256
    (one block row, s1 = 128 = c'), against the plain update with the same softmax approximation."""
    s0, c, cp = 256, 100, 128
    s1 = 32768 // s0
    steps = sorted(set(sm.rotation_steps(c, s1)) | set(mx.rotation_steps("abt", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1)) |
                   set(mx.rotation_steps("atb", cp, s0, s1, pru=True)))
    note("config 3 context + keys (%d rotations)" % len(steps))
    ctx, sk, keys = make_gpu("n16l12", seed=2700, rot_steps=steps)
    X = np.hstack([inputs.features(1003, 256, 768), np.ones((256, 1))])
    Y = np.eye(c)[inputs.labels(1003, 256, c)]
    W = inputs.weights(1003, c, 769)
    V = inputs.weights(1004, c, 769)

    def enc(M, tiling, seed):
        nb = int(np.prod(ctx.mat_blocks(M.shape[0], M.shape[1], s0, tiling, cp)))
        r = [inputs.encryption_randomness(seed, b, ctx.q[:12], ctx.n) for b in range(nb)]
        return ctx.mat_encrypt(sk, M, s0, 11, 2.0 ** 40, np.stack([x[0] for x in r]), np.stack([x[1] for x in r]),
                               tiling=tiling, c=cp)
    gx, gy, gw, gv = enc(X, 0, 301), enc(Y, 2, 302), enc(W, 1, 303), enc(V, 1, 304)
    lr, gamma = 1.0 / 256, tr.nag_gamma(2)
    note("config 3 step")
    gr = ctx.refresher(sk, lambda i: inputs.refresh_randomness(2701, i, ctx.q, ctx.n))
    gW, gV, nref = ctx.nag_step(keys, gx, gy, gw, gv, c, lr, gamma, refresh=gr)
    assert nref > 0
    prm = sm.SoftmaxParams()
    want_w, want_v = tr.nag_step_plain(X, Y, W, V, lr, gamma, lambda L: sm.asoftmax_rows(L, prm))
    assert np.abs(ctx.mat_decrypt(sk, gW)[:c, :769] - want_w).max() < 1e-4
    assert np.abs(ctx.mat_decrypt(sk, gV)[:c, :769] - want_v).max() < 1e-4
