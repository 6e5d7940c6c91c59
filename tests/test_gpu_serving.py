"""The request loop on the GPU (toy ring): two clients with their own seeded keys, two lanes (contexts on their own
streams).  A second round arrives while the first is still on the device (held there by a spin on its lane), is
admitted at once and runs on the other lane, finishing first; every served result equals the same product computed
alone, word for word."""
import sys

import pytest
import torch

from oracle import matrix as mx
from paper_2403_14111_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print("[case] serving: " + msg, file=sys.stderr, flush=True)


def test_requests_arriving_in_flight_overlap_and_equal_standalone_products():
    from paper_2403_14111_amd import hetal, serving
    s0, c = 16, 8
    steps = sorted(set(mx.rotation_steps("abt", c, s0, 128)) | set(mx.rotation_steps("atb", c, s0, 128)))
    note("context, two lanes, two clients")
    s_a, s_b = serving.concurrent_streams(2)             # lanes on streams of their own, on separate hardware queues
    with torch.cuda.stream(s_a):
        ctx = hetal.Context("toy")
    lanes = [ctx, ctx.share(s_b)]
    server = serving.Server(lanes, 1 << 34, free_memory=serving.torch_free_memory)
    assert all(not lane.tune_get("abt", c, s0, 4, 4)["two_streams"] for lane in lanes)
    data = {}
    for cl in (0, 1):
        sk = ctx.keygen(4100 + cl)
        keys = ctx.keys_create()
        keys.gen_evk(sk, 4100 + cl, rot_steps=steps, conj=True, relin=True)
        server.add_client(cl, keys)
        X = inputs.toy_matrix(7000 + cl, 16, 40, 0)
        W = inputs.toy_matrix(7000 + cl, 6, 40, 1)
        P = inputs.toy_matrix(7100 + cl, 16, 6, 0)
        data[cl] = (ctx.mat_encrypt_seeded(sk, X, s0, 4, 2.0 ** 40, 4100 + cl, 0),
                    ctx.mat_encrypt_seeded(sk, W, s0, 4, 2.0 ** 40, 4100 + cl, 10, tiling=1, c=c),
                    ctx.mat_encrypt_seeded(sk, P, s0, 4, 2.0 ** 40, 4100 + cl, 20, tiling=2, c=c))

    def reqs_of(cl, first):
        gx, gw, gp = data[cl]
        out = []
        for i in range(6):
            if i % 3 == 2:
                out.append(serving.Request(first + i, cl, "atb", gp, gx, c, 0.5))
            else:
                out.append(serving.Request(first + i, cl, "abt", gx, gw, c, 1.0 + i))
        return out

    note("warm-up: masks encoded on both lanes")
    for lane in lanes:
        with torch.cuda.stream(lane.stream):
            for cl in (0, 1):
                lane.enc_matmul_batch(server.keys[cl], [(r.op, r.a, r.b, r.c, r.t) for r in reqs_of(cl, 0)])
    torch.cuda.synchronize()

    note("round 1 behind a spin on lane 0, round 2 while it is in flight")
    with torch.cuda.stream(lanes[0].stream):
        torch.cuda._sleep(100_000_000)                   # tens of ms of spinning: round 1 stays in flight
    first = reqs_of(0, 0)
    for r in first:
        server.submit(r)
    server.step()
    assert [g.lane for g in server.inflight] == [0]
    second = reqs_of(1, 100)
    for r in second:
        server.submit(r)
    server.step()
    assert server.rounds[1][3] == 6                      # admitted with round 1's six requests in flight
    assert all(r.lane == 1 for r in second)
    finished = []
    while server.inflight:
        finished += server.step()
    assert sorted(r.rid for r in finished) == [r.rid for r in first + second]
    assert max(r.done for r in second) < min(r.done for r in first)   # round 2 overlapped and finished first
    note("results against standalone products")
    with torch.cuda.stream(ctx.stream):
        alones = [ctx.enc_matmul_abt(server.keys[r.client], r.a, r.b, r.c, r.t) if r.op == "abt"
                  else ctx.enc_matmul_atb(server.keys[r.client], r.a, r.b, r.c, r.t) for r in finished]
    torch.cuda.synchronize()
    for r, alone in zip(finished, alones):
        w = alone.n_rb * alone.n_cb * ctx.ct_words(alone.level)
        assert r.result.level == alone.level and r.result.scale == alone.scale
        assert torch.equal(r.result.buf[:w], alone.buf[:w]), r.rid
