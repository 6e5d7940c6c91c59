"""Batched products recorded into a HIP graph (hetal_enc_matmul_batch_graph): every replay equals the eager
batch word for word, with other eager work and cleared outputs between replays, and a replay after the inputs'
contents change recomputes from the new contents."""
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
    print("[case] graph " + msg, file=sys.stderr, flush=True)


def words(ctx, m):
    return m.buf[:m.n_rb * m.n_cb * ctx.ct_words(m.level)].clone()


def test_graph_replays_equal_the_eager_batch():
    s0, s1, c = 16, 128, 8
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        steps = sorted(set(mx.rotation_steps("abt", c, s0, s1)) | set(mx.rotation_steps("atb", c, s0, s1)))
        note("toy context on a created stream")
        ctx, sk, keys = make_gpu("toy", seed=2004, rot_steps=steps)

        def enc(mat, tiling, seed):
            return enc_mat_gpu(ctx, sk, mat, s0, 4, tiling, c, seed)[0]
        A = enc(inputs.toy_matrix(6300, 16, 40, 0), 0, 64)
        B = enc(inputs.toy_matrix(6300, 8, 40, 1), 1, 65)
        P = enc(inputs.toy_matrix(6301, 16, 8, 0), 2, 66)
        A2 = enc(inputs.toy_matrix(6302, 16, 40, 0), 0, 67)
        reqs = [("abt", A, B, c, 1.0), ("atb", P, A, c, 0.5)]
        eager = [words(ctx, m) for m in ctx.enc_matmul_batch(keys, reqs)]
        note("capture")
        outs, graph = ctx.enc_matmul_batch_graph(keys, reqs)
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(words(ctx, o), e)
        for rep in range(3):
            note("replay %d" % rep)
            for o in outs:
                o.buf.zero_()
            ctx.enc_matmul_abt(keys, A2, B, c, -1.0)           # other work on the same pools in between
            graph.launch()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                assert torch.equal(words(ctx, o), e), rep
        note("replay on new input contents")
        A.buf.copy_(A2.buf)
        graph.launch()
        want = [words(ctx, m) for m in ctx.enc_matmul_batch(keys, [("abt", A2, B, c, 1.0), ("atb", P, A2, c, 0.5)])]
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            assert torch.equal(words(ctx, o), w)
        assert not torch.equal(want[0], eager[0])
        del graph
        torch.cuda.synchronize()
