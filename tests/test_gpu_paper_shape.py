"""GPU parity at a shape of the paper's Table 4 on the benchmark ring (N = 2^16, 12 + 3 primes, dnum = 4):
(a, b, c) = (128, 128, 4) with s0 = a = 128, s1 = 256.  DiagABT (Alg. 1), DiagATB on the RotLeft branch
(level(A) >= level(B), Alg. 2) and on the PRotUp branch (level(A) < level(B), Alg. 3), each compared word for word
with the oracle, decrypted within 2^-18 of FP64, and with the operation counts of Table matnum_fixed."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import make_gpu
from tests.oracle_setup import make_oracle
from tests.test_gpu_parity import TARGET, compare_blocks, enc_mat_both

pytestmark = pytest.mark.gpu

A_ROWS, B_COLS, C, LEVEL = 128, 128, 4, 11
S0 = A_ROWS
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def note(msg):
    print("[case] paper-shape (128,128,4) " + msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def shape():
    s1 = 32768 // S0
    steps = sorted(set(mx.rotation_steps("abt", C, S0, s1)) | set(mx.rotation_steps("atb", C, S0, s1)) |
                   set(mx.rotation_steps("atb", C, S0, s1, pru=True)))
    note("context + keys (%d rotations), GPU and oracle" % len(steps))
    ctx, sk, keys = make_gpu("n16l12", seed=2004, rot_steps=steps)
    ev = make_oracle("n16l12", seed=2004, rot_steps=steps)
    A = inputs.toy_matrix(1128, A_ROWS, B_COLS, 0)
    B = inputs.toy_matrix(1128, C, B_COLS, 1)
    P = inputs.toy_matrix(1129, A_ROWS, C, 0)
    row = [r for r in json.load(open(os.path.join(GOLDEN, "matnum_fixed.json")))["rows"]
           if (r["a"], r["b"], r["c"]) == (A_ROWS, B_COLS, C)][0]
    return ctx, sk, keys, ev, (A, B, P), s1, row


def counted(ctx, run):
    import torch
    torch.cuda.synchronize()
    ctx.reset_counters()
    out = run()
    torch.cuda.synchronize()
    return out, ctx.counters()


def test_diag_abt_bit_exact_with_table_counts(shape):
    ctx, sk, keys, ev, (A, B, P), s1, row = shape
    note("DiagABT")
    ga, oa = enc_mat_both(ctx, sk, ev, A, S0, LEVEL, 0, C, seed=51)
    gb, ob = enc_mat_both(ctx, sk, ev, B, S0, LEVEL, 1, C, seed=52)
    gout, ops = counted(ctx, lambda: ctx.enc_matmul_abt(keys, ga, gb, C, 1.0))
    assert {k: ops[k] for k in ("cmult", "mult", "rot")} == row["abt"]
    oout = mx.diag_abt(ev, oa, ob[0], C, S0, s1, 1.0)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    assert np.abs(res[:A_ROWS, :s1] - np.tile(A @ B.T, (1, s1 // C))).max() < TARGET


@pytest.mark.parametrize("branch", ["rl", "pru"])
def test_diag_atb_bit_exact_with_table_counts(shape, branch):
    ctx, sk, keys, ev, (A, B, P), s1, row = shape
    note("DiagATB %s" % branch)
    la = LEVEL if branch == "rl" else LEVEL - 1
    gp, op_ = enc_mat_both(ctx, sk, ev, P, S0, la, 2, C, seed=53)
    ga, oa = enc_mat_both(ctx, sk, ev, A, S0, LEVEL, 0, C, seed=54)
    gout, ops = counted(ctx, lambda: ctx.enc_matmul_atb(keys, gp, ga, C, 1.0))
    want = row["atb_" + branch]
    assert {k: ops[k] for k in want} == want
    oout = mx.diag_atb(ev, op_, oa, C, S0, s1, 1.0)
    compare_blocks(ctx, gout, oout)
    res = ctx.mat_decrypt(sk, gout)
    assert np.abs(res[:S0, :B_COLS] - np.tile(P.T @ A, (S0 // C, 1))).max() < TARGET
