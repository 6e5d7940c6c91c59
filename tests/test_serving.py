"""The request loop's scheduling logic on the CPU, with a stand-in context that records its batched calls."""
import numpy as np
import pytest

from paper_2403_14111_amd import serving


class FakeMat:
    def __init__(self, n_rb, n_cb, level):
        self.n_rb, self.n_cb, self.level = n_rb, n_cb, level


class FakeCtx:
    def __init__(self, clock=None, cost=0.01):
        self.calls = []
        self.clock = clock
        self.cost = cost

    def ct_words(self, level):
        return 2 * (level + 1) * 1024

    def enc_matmul_batch(self, keys, reqs):
        self.calls.append((keys, [(op, a, b, c, t) for op, a, b, c, t in reqs]))
        if self.clock is not None:
            self.clock.t += self.cost * len(reqs)
        return ["out:%s:%d" % (keys, i) for i in range(len(reqs))]


class FakeClock:
    def __init__(self):
        self.t = 100.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def req(rid, client, op="abt", blocks=1, level=11, arrival=0.0):
    a = FakeMat(blocks, 1, level) if op == "abt" else FakeMat(1, 1, level)
    b = FakeMat(1, 1, level) if op == "abt" else FakeMat(1, blocks, level)
    return serving.Request(rid, client, op, a, b, 16, 1.0, arrival)


def test_admission_takes_the_queue_head_in_order_within_the_budget():
    ctx = FakeCtx()
    sizes = [serving.request_bytes(ctx, req(i, "x", blocks=1 + i % 3)) for i in range(6)]
    budget = sizes[0] + sizes[1] + sizes[2] // 2
    srv = serving.Server(ctx, budget)
    srv.add_client("x", "kx")
    for i in range(6):
        srv.submit(req(i, "x", blocks=1 + i % 3))
    first = srv.admit()
    assert [r.rid for r in first] == [0, 1]           # the third would exceed the budget
    assert [r.rid for r in srv.queue] == [2, 3, 4, 5]  # order kept


def test_a_request_larger_than_the_budget_still_runs_alone():
    ctx = FakeCtx()
    srv = serving.Server(ctx, 1)
    srv.add_client("x", "kx")
    srv.submit(req(0, "x", blocks=4))
    srv.submit(req(1, "x"))
    assert [r.rid for r in srv.admit()] == [0]
    assert [r.rid for r in srv.admit()] == [1]


def test_one_batched_call_per_client_per_round_in_arrival_order():
    ctx = FakeCtx()
    srv = serving.Server(ctx, 1 << 60)
    srv.add_client("x", "kx")
    srv.add_client("y", "ky")
    order = ["y", "x", "y", "y", "x"]
    for i, cl in enumerate(order):
        srv.submit(req(i, cl, op="abt" if i % 2 else "atb"))
    done = srv.step()
    assert [r.rid for r in done] == [0, 1, 2, 3, 4]
    assert [k for k, _ in ctx.calls] == ["ky", "kx"]   # first queued client first
    assert [r[0] for r in ctx.calls[0][1]] == ["atb", "atb", "abt"]
    assert all(r.result is not None and r.done is not None for r in done)
    assert srv.rounds[0][1:] == (5, 2)


def test_unknown_client_is_rejected():
    srv = serving.Server(FakeCtx(), 1 << 30)
    with pytest.raises(KeyError):
        srv.submit(req(0, "nobody"))


def test_replay_batches_what_arrived_and_measures_latency():
    clock = FakeClock()
    ctx = FakeCtx(clock=clock, cost=0.010)
    srv = serving.Server(ctx, 1 << 60, clock=clock)
    srv.add_client("x", "kx")
    # three at t=0 (one round of 3), one at 0.005 (arrives while that round runs), one at 1.0 (alone)
    reqs = [req(i, "x", arrival=a) for i, a in enumerate([0.0, 0.0, 0.0, 0.005, 1.0])]
    finished = serving.serve(srv, reqs, clock=clock, sleep=clock.sleep)
    assert sorted(r.rid for r in finished) == [0, 1, 2, 3, 4]
    assert [n for _, n, _ in srv.rounds] == [3, 1, 1]
    lat = {r.rid: r.latency for r in finished}
    assert lat[0] == pytest.approx(0.030)            # waited for nothing, 3 requests x 10 ms
    assert lat[3] == pytest.approx(0.030 - 0.005 + 0.010)
    assert lat[4] == pytest.approx(0.010)


def test_poisson_arrivals_are_increasing_with_the_right_mean_gap():
    rng = np.random.default_rng(5)
    t = serving.poisson_arrivals(rng, 50.0, 4000)
    assert len(t) == 4000 and all(b > a for a, b in zip(t, t[1:]))
    assert np.mean(np.diff([0.0] + t)) == pytest.approx(1 / 50.0, rel=0.05)


def test_latency_summary_percentiles():
    rs = []
    for i in range(100):
        r = serving.Request(i, "x", "abt", None, None, 16, arrival=float(i))
        r.done = float(i) + (i + 1) / 1000.0
        rs.append(r)
    s = serving.latency_summary(rs, 1.0)
    assert s["latency_ms_p50"] == pytest.approx(51.0, abs=1.0)
    assert s["latency_ms_p99"] == pytest.approx(99.0, abs=1.0)
    assert s["latency_ms_max"] == pytest.approx(100.0)
