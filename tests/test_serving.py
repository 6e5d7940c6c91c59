"""The request loop's scheduling logic on the CPU, with stand-in contexts (lanes) whose batched calls take time on a
fake clock and whose events complete when their lane has worked through what was queued before them."""
import numpy as np
import pytest

from paper_2403_14111_amd import serving


class FakeMat:
    def __init__(self, n_rb, n_cb, level):
        self.n_rb, self.n_cb, self.level = n_rb, n_cb, level


class FakeClock:
    def __init__(self):
        self.t = 100.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeLane:
    """A context on its own stream: work queued on it runs back to back, `cost` seconds per request."""

    def __init__(self, name, clock, cost=0.01):
        self.name, self.clock, self.cost = name, clock, cost
        self.calls = []
        self.busy_until = 0.0

    def ct_words(self, level):
        return 2 * (level + 1) * 1024

    def enc_matmul_batch(self, keys, reqs):
        self.calls.append((keys, [(op, a, b, c, t) for op, a, b, c, t in reqs]))
        self.busy_until = max(self.busy_until, self.clock()) + self.cost * len(reqs)
        return ["out:%s:%s:%d" % (self.name, keys, i) for i in range(len(reqs))]


class FakeEvent:
    def __init__(self, clock, at):
        self.clock, self.at = clock, at

    def query(self):
        return self.clock() >= self.at

    def synchronize(self):
        self.clock.t = max(self.clock.t, self.at)


def make_server(lanes=1, budget=1 << 60, cost=0.01, free=None):
    clock = FakeClock()
    ls = [FakeLane("L%d" % i, clock, cost) for i in range(lanes)]
    srv = serving.Server(ls, budget, clock=clock, record=lambda lane: FakeEvent(clock, lane.busy_until),
                         run=lambda lane, fn: fn(), free_memory=free, margin=0)
    return srv, ls, clock


def req(rid, client, op="abt", blocks=1, level=11, arrival=0.0):
    a = FakeMat(blocks, 1, level) if op == "abt" else FakeMat(1, 1, level)
    b = FakeMat(1, 1, level) if op == "abt" else FakeMat(1, blocks, level)
    return serving.Request(rid, client, op, a, b, 16, 1.0, arrival)


def size(r):
    return serving.request_bytes(FakeLane("x", FakeClock()), r)


def test_admission_takes_the_queue_head_in_order_within_the_budget():
    sizes = [size(req(i, "x", blocks=1 + i % 3)) for i in range(6)]
    srv, _, _ = make_server(budget=sizes[0] + sizes[1] + sizes[2] // 2)
    srv.add_client("x", "kx")
    for i in range(6):
        srv.submit(req(i, "x", blocks=1 + i % 3))
    first = srv.admit()
    assert [r.rid for r in first] == [0, 1]           # the third would exceed the budget
    assert [r.rid for r in srv.queue] == [2, 3, 4, 5]  # order kept


def test_a_request_larger_than_the_budget_still_runs_alone():
    srv, _, clock = make_server(budget=1)
    srv.add_client("x", "kx")
    srv.submit(req(0, "x", blocks=4))
    srv.submit(req(1, "x"))
    srv.step()
    assert [r.rid for g in srv.inflight for r in g.reqs] == [0]
    srv.step()                                          # 0 still running: 1 does not fit beside it
    assert [r.rid for r in srv.queue] == [1]
    clock.t += 1.0
    done = srv.step()                                   # 0 finishes, then 1 is admitted alone
    assert [r.rid for r in done] == [0] and [r.rid for g in srv.inflight for r in g.reqs] == [1]


def test_requests_are_admitted_while_others_are_in_flight():
    srv, lanes, clock = make_server(lanes=2)
    srv.add_client("x", "kx")
    srv.add_client("y", "ky")
    for i in range(3):
        srv.submit(req(i, "x"))
    srv.step()
    assert srv.inflight and not srv.queue
    clock.t += 0.005                                    # the first round is still running
    srv.submit(req(3, "y"))
    srv.submit(req(4, "x"))
    srv.step()
    assert srv.rounds[1][3] == 3                         # three requests in flight when the second round started
    assert len(srv.inflight) == 3
    # the second round's groups went to the less loaded lanes: y to the idle lane 1, then x to lane 1 as well
    # (lane 0 still holds the first round's three requests)
    assert [k for k, _ in lanes[0].calls] == ["kx"] and [k for k, _ in lanes[1].calls] == ["ky", "kx"]


def test_memory_reservations_hold_until_completion():
    one = size(req(0, "x"))
    srv, _, clock = make_server(budget=2 * one)
    srv.add_client("x", "kx")
    for i in range(4):
        srv.submit(req(i, "x"))
    srv.step()
    assert srv.reserved == 2 * one and [r.rid for r in srv.queue] == [2, 3]
    assert srv.step() == [] and srv.reserved == 2 * one   # nothing finished, nothing admitted
    clock.t += 1.0
    done = srv.step()
    assert [r.rid for r in done] == [0, 1] and srv.reserved == 2 * one and not srv.queue


def test_free_device_memory_limits_admission():
    one = size(req(0, "x"))
    free = [10 * one]
    srv, _, clock = make_server(free=lambda: free[0])
    srv.add_client("x", "kx")
    srv.submit(req(0, "x"))
    srv.step()
    free[0] = one // 2                                   # the device filled up meanwhile
    srv.submit(req(1, "x"))
    srv.step()
    assert [r.rid for r in srv.queue] == [1]
    clock.t += 1.0
    free[0] = 10 * one
    srv.step()
    assert not srv.queue


def test_one_batched_call_per_client_per_round_in_arrival_order():
    srv, lanes, clock = make_server()
    srv.add_client("x", "kx")
    srv.add_client("y", "ky")
    order = ["y", "x", "y", "y", "x"]
    for i, cl in enumerate(order):
        srv.submit(req(i, cl, op="abt" if i % 2 else "atb"))
    srv.step()
    assert [k for k, _ in lanes[0].calls] == ["ky", "kx"]   # first queued client first
    assert [r[0] for r in lanes[0].calls[0][1]] == ["atb", "atb", "abt"]
    clock.t += 1.0
    done = srv.step()
    assert sorted(r.rid for r in done) == [0, 1, 2, 3, 4]
    assert all(r.result is not None and r.done == clock.t for r in done)
    assert srv.rounds[0][1:3] == (5, 2)


def test_unknown_client_is_rejected():
    srv, _, _ = make_server()
    with pytest.raises(KeyError):
        srv.submit(req(0, "nobody"))


def test_replay_overlaps_rounds_and_measures_latency():
    srv, lanes, clock = make_server(lanes=2, cost=0.010)
    srv.add_client("x", "kx")
    srv.add_client("y", "ky")
    # three at t=0 (x), one at 0.005 (y: admitted at once on the idle lane), one at 1.0 (alone)
    reqs = [req(0, "x"), req(1, "x"), req(2, "x"), req(3, "y", arrival=0.005), req(4, "x", arrival=1.0)]
    finished = serving.serve(srv, reqs, clock=clock, sleep=clock.sleep, idle=1e-4)
    assert sorted(r.rid for r in finished) == [0, 1, 2, 3, 4]
    lat = {r.rid: r.latency for r in finished}
    assert lat[0] == pytest.approx(0.030, abs=2e-4)      # 3 requests x 10 ms on lane 0
    assert lat[3] == pytest.approx(0.010, abs=2e-4)      # ran beside them on lane 1, not after them
    assert lat[4] == pytest.approx(0.010, abs=2e-4)
    assert {r.rid: r.lane for r in finished}[3] == 1


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


def test_several_lanes_keep_to_their_own_streams():
    class Lane(FakeLane):
        two = True

        def set_two_streams(self, on):
            self.two = on
    clock = FakeClock()
    one = Lane("solo", clock)
    serving.Server([one], 1 << 40, clock=clock)
    assert one.two                                    # a single lane may still use its second stream
    ls = [Lane("a", clock), Lane("b", clock)]
    serving.Server(ls, 1 << 40, clock=clock)
    assert not any(lane.two for lane in ls)


def test_a_failing_batched_call_hands_its_requests_back_with_the_error():
    class Boom(FakeLane):
        def enc_matmul_batch(self, keys, reqs):
            if keys == "kbad":
                raise RuntimeError("E_SHAPE: bad request")
            return super().enc_matmul_batch(keys, reqs)
    clock = FakeClock()
    lane = Boom("L0", clock)
    srv = serving.Server([lane], 1 << 60, clock=clock, record=lambda ln: FakeEvent(clock, ln.busy_until),
                         run=lambda ln, fn: fn(), margin=0)
    srv.add_client("good", "kgood")
    srv.add_client("bad", "kbad")
    srv.submit(req(0, "bad"))
    srv.submit(req(1, "good"))
    first = srv.step()
    assert [r.rid for r in first] == [0] and isinstance(first[0].error, RuntimeError) and first[0].result is None
    assert srv.reserved == size(req(1, "good"))      # only the good group holds memory
    clock.t += 1.0
    done = srv.step()
    assert [r.rid for r in done] == [1] and done[0].error is None and srv.reserved == 0
    s = serving.latency_summary(first + done, 1.0)
    assert s["requests"] == 1 and s["errors"] == 1
