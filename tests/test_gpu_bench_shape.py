"""GPU parity at the benchmark's exact workload: the forward product X W^T (X 128 x 768, W 10 x 768 -> c = 16)
and the gradient product (P - Y)^T X, N = 2^16, 12 + 3 primes, inputs at level 11, s0 = 128 -- every output word
against the oracle (the oracle takes tens of seconds here)."""
import sys

import numpy as np
import pytest

from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import make_gpu
from tests.oracle_setup import make_oracle
from tests.test_gpu_parity import TARGET, compare_blocks, enc_mat_both

pytestmark = pytest.mark.gpu

S0, C, LEVEL = 128, 16, 11


def note(msg):
    print("[case] bench-shape " + msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    s1 = 32768 // S0
    steps = sorted(set(mx.rotation_steps("abt", C, S0, s1)) | set(mx.rotation_steps("atb", C, S0, s1)))
    note("context + keys (%d rotations), GPU and oracle" % len(steps))
    ctx, sk, keys = make_gpu("n16l12", seed=2000, rot_steps=steps)
    ev = make_oracle("n16l12", seed=2000, rot_steps=steps)
    X = inputs.features(1002, 128, 768)
    W = inputs.weights(1002, 10, 768)
    PY = inputs.softmax_minus_onehot(X @ W.T, inputs.labels(1002, 128, 10), 10)
    note("encrypt")
    gx, ox = enc_mat_both(ctx, sk, ev, X, S0, LEVEL, 0, C, seed=3000)
    gw, ow = enc_mat_both(ctx, sk, ev, W, S0, LEVEL, 1, C, seed=3100)
    gpy, opy = enc_mat_both(ctx, sk, ev, PY, S0, LEVEL, 2, C, seed=3200)
    return ctx, sk, keys, ev, (X, W, PY), (gx, gw, gpy), (ox, ow, opy), s1


_ORACLE = {}


def oracle_product(setup, op):
    """The oracle's output of one product, computed once per module (tens of seconds each)."""
    ctx, sk, keys, ev, _, _, (ox, ow, opy), s1 = setup
    if op not in _ORACLE:
        note("%s 128x768x10 in the oracle" % op)
        _ORACLE[op] = (mx.diag_abt(ev, ox, ow[0], C, S0, s1, 1.0) if op == "abt"
                       else mx.diag_atb(ev, opy, ox, C, S0, s1, 1.0))
    return _ORACLE[op]


def test_forward_product_bit_exact(setup):
    ctx, sk, keys, ev, (X, W, PY), (gx, gw, gpy), (ox, ow, opy), s1 = setup
    note("DiagABT 128x768x10 on the GPU")
    gout = ctx.enc_matmul_abt(keys, gx, gw, C, 1.0)
    oout = oracle_product(setup, "abt")
    compare_blocks(ctx, gout, oout)
    Wp = np.vstack([W, np.zeros((C - 10, 768))])
    res = ctx.mat_decrypt(sk, gout)[:128, :s1]
    assert np.abs(res - np.tile(X @ Wp.T, (1, s1 // C))).max() < TARGET


def test_gradient_product_bit_exact(setup):
    ctx, sk, keys, ev, (X, W, PY), (gx, gw, gpy), (ox, ow, opy), s1 = setup
    note("DiagATB (128x10)^T 128x768 on the GPU")
    gout = ctx.enc_matmul_atb(keys, gpy, gx, C, 1.0)
    oout = oracle_product(setup, "atb")
    compare_blocks(ctx, gout, oout)
    PYp = np.hstack([PY, np.zeros((128, C - 10))])
    res = ctx.mat_decrypt(sk, gout)[:S0, :768]
    assert np.abs(res - np.tile(PYp.T @ X, (S0 // C, 1))).max() < TARGET


def test_benchmark_launch_configuration_bit_exact(setup):
    """Both products as the benchmark times them: one batched call whose two products run on two streams,
    repeated, every output word against the oracle each time."""
    ctx, sk, keys, ev, _, (gx, gw, gpy), _, s1 = setup
    for rep in range(2):
        note("batched two-stream call, repetition %d" % rep)
        gabt, gatb = ctx.enc_matmul_batch(keys, [("abt", gx, gw, C, 1.0), ("atb", gpy, gx, C, 1.0)])
        compare_blocks(ctx, gabt, oracle_product(setup, "abt"))
        compare_blocks(ctx, gatb, oracle_product(setup, "atb"))
