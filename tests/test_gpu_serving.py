"""The request loop on the GPU (toy ring): two clients with their own keys, requests of both kinds arriving in a
burst; every served result must equal the same product computed alone, word for word."""
import sys

import pytest
import torch

from oracle import matrix as mx
from paper_2403_14111_amd import inputs
from tests.gpu_setup import make_gpu
from tests.test_gpu_parity import enc_mat_gpu

pytestmark = pytest.mark.gpu


def test_served_results_equal_standalone_products():
    from paper_2403_14111_amd import serving
    print("[case] serving: two clients, twelve requests", file=sys.stderr, flush=True)
    s0, c = 16, 8
    steps = sorted(set(mx.rotation_steps("abt", c, s0, 128)) | set(mx.rotation_steps("atb", c, s0, 128)))
    ctx, sk0, keys0 = make_gpu("toy", seed=2100, rot_steps=steps)
    clients = {0: (sk0, keys0), 1: make_keys(ctx, 2101, steps)}
    server = serving.Server(ctx, 1 << 34, sync=torch.cuda.synchronize)
    data = {}
    for cl, (sk, keys) in clients.items():
        server.add_client(cl, keys)
        X = inputs.toy_matrix(7000 + cl, 16, 40, 0)
        W = inputs.toy_matrix(7000 + cl, 6, 40, 1)
        P = inputs.toy_matrix(7100 + cl, 16, 6, 0)
        data[cl] = (enc_mat_gpu(ctx, sk, X, s0, 4, 0, c, 90 + cl)[0], enc_mat_gpu(ctx, sk, W, s0, 4, 1, c, 92 + cl)[0],
                    enc_mat_gpu(ctx, sk, P, s0, 4, 2, c, 94 + cl)[0])
    reqs = []
    for i in range(12):
        cl = [0, 1, 1, 0, 0, 1, 0, 1, 1, 1, 0, 0][i]
        gx, gw, gp = data[cl]
        if i % 3 == 2:
            reqs.append(serving.Request(i, cl, "atb", gp, gx, c, 0.5, 0.0))
        else:
            reqs.append(serving.Request(i, cl, "abt", gx, gw, c, 1.0 + i, 0.0))
    finished = serving.serve(server, reqs)
    assert sorted(r.rid for r in finished) == list(range(12))
    assert len(server.rounds) == 1 and server.rounds[0][1:] == (12, 2)
    for r in finished:
        alone = (ctx.enc_matmul_abt(server.keys[r.client], r.a, r.b, r.c, r.t) if r.op == "abt"
                 else ctx.enc_matmul_atb(server.keys[r.client], r.a, r.b, r.c, r.t))
        w = alone.n_rb * alone.n_cb * ctx.ct_words(alone.level)
        assert r.result.level == alone.level and r.result.scale == alone.scale
        assert torch.equal(r.result.buf[:w], alone.buf[:w]), r.rid


def make_keys(ctx, seed, steps):
    """A second client's secret and keys in an existing context."""
    sk = ctx.sk_create(inputs.ternary_secret(seed, ctx.n))
    keys = ctx.keys_create()
    a, e = inputs.switch_key_randomness(seed, inputs.key_id(0), ctx.dnum, ctx.primes, ctx.n)
    keys.gen_relin(sk, a, e)
    for g in sorted(set(ctx.galois_rot(r) for r in steps) | {ctx.galois_conj()}):
        a, e = inputs.switch_key_randomness(seed, inputs.key_id(1, g), ctx.dnum, ctx.primes, ctx.n)
        keys.gen_galois(sk, g, a, e)
    return sk, keys
