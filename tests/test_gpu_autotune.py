"""The schedule choices of the batched products and their autotuner: every choice leaves every output word
unchanged.  Toy ring: a mixed batch (DiagABT, DiagATB on both branches) under the tuner and under forced extreme
choices -- working-set limits down to one ciphertext, so that the products run in many chunks and every lockstep
group splits -- against the defaults; full ring: one product under each conversion-task size and launch group
size."""
import sys

import numpy as np
import pytest
import torch

from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import make_gpu
from tests.test_gpu_parity import enc_mat_gpu

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] autotune " + msg, file=sys.stderr, flush=True)


def words(ctx, m):
    return m.buf[:m.n_rb * m.n_cb * ctx.ct_words(m.level)]


def assert_same(ctx, xs, ys):
    for x, y in zip(xs, ys):
        assert (x.n_rb, x.n_cb, x.level, x.scale) == (y.n_rb, y.n_cb, y.level, y.scale)
        assert torch.equal(words(ctx, x), words(ctx, y))


def test_tuner_and_forced_schedules_leave_results_unchanged():
    s0 = 16
    steps = sorted(set(mx.rotation_steps("abt", 8, s0, 128)) | set(mx.rotation_steps("abt", 4, s0, 128)) |
                   set(mx.rotation_steps("atb", 8, s0, 128, pru=True)))
    note("toy batch")
    ctx, sk, keys = make_gpu("toy", seed=2200, rot_steps=steps)
    reqs = []
    for n, (ar, ac, br, c) in enumerate([(16, 32, 8, 8), (40, 300, 7, 8), (16, 32, 3, 4)]):
        A = inputs.toy_matrix(8000 + n, ar, ac, 0)
        B = inputs.toy_matrix(8000 + n, br, ac, 1)
        reqs.append(("abt", enc_mat_gpu(ctx, sk, A, s0, 4, 0, c, 300 + n)[0],
                     enc_mat_gpu(ctx, sk, B, s0, 4, 1, c, 310 + n)[0], c, 1.0))
    for n, (rows, cols) in enumerate([(16, 32), (30, 150)]):
        P = inputs.toy_matrix(8100 + n, rows, 8, 0)
        X = inputs.toy_matrix(8100 + n, rows, cols, 1)
        reqs.append(("atb", enc_mat_gpu(ctx, sk, P, s0, 4, 2, 8, 320 + n)[0],
                     enc_mat_gpu(ctx, sk, X, s0, 4, 0, 8, 330 + n)[0], 8, 0.5))
        # the same shapes with Abar a level lower: the PRotUp branch
        reqs.append(("atb", enc_mat_gpu(ctx, sk, P, s0, 3, 2, 8, 340 + n)[0],
                     enc_mat_gpu(ctx, sk, X, s0, 4, 0, 8, 350 + n)[0], 8, 0.5))
    classes = (("abt", 8, s0, 4, 4), ("abt", 4, s0, 4, 4), ("atb", 8, s0, 4, 4), ("atb", 8, s0, 3, 4))
    ref = ctx.enc_matmul_batch(keys, reqs)
    tuned, rep = ctx.autotune_batch(keys, reqs, reps=1)
    assert rep["classes"] == 4 and rep["trials"] >= 4 * 12
    assert_same(ctx, tuned, ref)
    assert_same(ctx, ctx.enc_matmul_batch(keys, reqs), ref)      # with the tuner's choices in place
    for cls in classes:
        t = ctx.tune_get(*cls)
        assert 1 <= t["ks_group"] <= 32 and t["tpt_modup"] >= 0 and t["tpt_moddown"] >= 0
    for ks_group, tpt_up, tpt_down, two, work in ((1, 1, 1, False, 1), (3, 2, 5, True, 5), (32, 100, 100, True, 0),
                                                  (7, 0, 0, True, 13)):
        note("forced schedule %s" % ((ks_group, tpt_up, tpt_down, two, work),))
        for cls in classes:
            ctx.tune_set(*cls, ks_group=ks_group, tpt_modup=tpt_up, tpt_moddown=tpt_down, two_streams=two,
                         work_cts=work)
        assert_same(ctx, ctx.enc_matmul_batch(keys, reqs), ref)
    # the single-product calls follow the defaults whatever a class was tuned to
    op, a, b, c, t = reqs[1]
    assert_same(ctx, [ctx.enc_matmul_abt(keys, a, b, c, t)], [ref[1]])
    ctx.tune_reset()
    assert ctx.tune_get("abt", 8, s0, 4, 4) == dict(ks_group=32, tpt_modup=0, tpt_moddown=0, two_streams=True,
                                                    work_cts=0)


@pytest.mark.parametrize("tpt", [1, 2, 5, 12])
def test_full_ring_conversion_tasks_and_groups(tpt):
    """N = 2^16: DiagABT of a 24 x 200 matrix (c = 16) under each conversion-task size, with launch groups of 3."""
    s0 = 128
    s1 = 32768 // s0
    note("full ring tpt=%d" % tpt)
    ctx, sk, keys = make_gpu("n16l12", seed=2201, rot_steps=mx.rotation_steps("abt", 16, s0, s1))
    A = inputs.toy_matrix(8200, 24, 200, 0)
    B = inputs.toy_matrix(8200, 10, 200, 1)
    ga = enc_mat_gpu(ctx, sk, A, s0, 11, 0, 16, 340)[0]
    gb = enc_mat_gpu(ctx, sk, B, s0, 11, 1, 16, 341)[0]
    ref = ctx.enc_matmul_batch(keys, [("abt", ga, gb, 16, 1.0)])
    ctx.tune_set("abt", 16, s0, 11, 11, ks_group=3, tpt_modup=tpt, tpt_moddown=tpt)
    assert_same(ctx, ctx.enc_matmul_batch(keys, [("abt", ga, gb, 16, 1.0)]), ref)
    res = ctx.mat_decrypt(sk, ref[0])
    Bp = np.vstack([B, np.zeros((6, 200))])
    assert np.abs(res[:24, :s1] - np.tile(A @ Bp.T, (1, s1 // 16))).max() < 2.0 ** -18
