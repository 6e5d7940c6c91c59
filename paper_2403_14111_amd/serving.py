"""A request loop for encrypted matrix products on one GPU, with continuous batching.

Clients submit DiagABT / DiagATB requests on ciphertexts already in device memory (block-encoded matrices made
with their own keys); every client's evaluation keys stay resident.  The server never waits for the device as a
whole:

  * admission: the queue's head is admitted, in arrival order, while the memory the admitted requests reserve fits
    the budget and the device's free memory (a callable, by default torch's view of HIP's free memory plus what
    its allocator holds unused) -- also while earlier requests are still running;
  * launch: the requests admitted together are grouped by client, and each group is one batched call
    (`enc_matmul_batch`, where requests sharing a shape class run in lockstep) on the least loaded lane -- a
    library context on a stream of its own (`Context.share`) -- so that groups of different rounds and clients
    run concurrently on the device.  HIP maps streams onto a few hardware queues when they are first used, and
    two streams on one queue run in turn: `concurrent_streams` picks lane streams that do run side by side, and
    with several lanes each keeps to its own stream (`Context.set_two_streams(False)`);
  * completion: an event recorded on the lane's stream after the group's work; a group is finished when its event
    is seen complete, and only then is its memory reservation released.

A request's result is the same ciphertext it would get alone: the batched call is bit-identical to single calls,
and the lanes share the keys and the parameters.
"""
import collections
import time


class Request:
    """One product: op "abt" (t A Bbar^T) or "atb" (t Abar^T B) on the client's matrices."""

    __slots__ = ("rid", "client", "op", "a", "b", "c", "t", "arrival", "start", "done", "result", "lane", "error")

    def __init__(self, rid, client, op, a, b, c, t=1.0, arrival=0.0):
        if op not in ("abt", "atb"):
            raise ValueError("op must be 'abt' or 'atb'")
        self.rid, self.client, self.op, self.a, self.b, self.c, self.t = rid, client, op, a, b, c, t
        self.arrival = arrival
        self.start = self.done = None
        self.result = None
        self.lane = None
        self.error = None  # the exception of a batched call that failed (then result stays None)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


def _shape(req):
    """(ciphertext level, run sums, products and rotations of the product loop, output blocks) of a request."""
    half = req.c // 2
    if req.op == "abt":
        level = min(req.a.level, req.b.level)
        runs = req.a.n_rb * half
        work = req.a.n_rb * req.a.n_cb * half + req.a.n_cb * half
        out_blocks = req.a.n_rb
    else:
        level = max(req.a.level, req.b.level)
        runs = (req.b.n_cb + req.a.n_rb) * half
        work = req.b.n_rb * req.b.n_cb * half * 3 + req.a.n_rb * half
        out_blocks = req.b.n_cb
    return level, runs, work, out_blocks


def request_bytes(ctx, req, work_limit=2 << 30):
    """Device memory a request holds while it runs, bounded from above: its run sums three times over (the sums,
    a rotated copy, the masked copy), one chunk of products and rotations (the library makes them at most
    `work_limit` bytes at a time), its result, and a margin for the level-dropped inputs."""
    level, runs, work, out_blocks = _shape(req)
    ct = ctx.ct_words(level) * 8
    return ct * (3 * runs + out_blocks + 40) + min(work * ct, work_limit)


def request_cost(req):
    """Relative device time of a request: its key switches (products, rotations, and the column or row sums)."""
    level, runs, work, _ = _shape(req)
    return (work + 2 * runs) * (level + 1)


def torch_free_memory():
    """Bytes the device can still hand out: HIP's free memory plus what torch's caching allocator holds unused."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    return free + torch.cuda.memory_reserved() - torch.cuda.memory_allocated()


class _Group:
    __slots__ = ("reqs", "event", "bytes", "lane", "cost")

    def __init__(self, reqs, event, nbytes, lane, cost):
        self.reqs, self.event, self.bytes, self.lane, self.cost = reqs, event, nbytes, lane, cost


class Server:
    """Continuous batching over a FIFO queue, with per-client keys, admission by memory, and several lanes.

    lanes: library contexts, each on its own stream (the first is the one the keys were made with; the others
    from `Context.share`).  record(lane) returns an event recorded on the lane's stream after the work queued so
    far, with .query() (done?) and .synchronize(); run(lane, fn) calls fn with the lane's stream current (so that
    the outputs are allocated for it).  free_memory() -> bytes, or None to admit by the budget alone."""

    def __init__(self, lanes, memory_budget, clock=time.perf_counter, record=None, run=None, free_memory=None,
                 margin=1 << 30, max_requests_per_round=256):
        self.lanes = list(lanes) if isinstance(lanes, (list, tuple)) else [lanes]
        self.ctx = self.lanes[0]
        if len(self.lanes) > 1:
            for lane in self.lanes:
                if hasattr(lane, "set_two_streams"):
                    lane.set_two_streams(False)
        self.memory_budget = memory_budget
        self.clock = clock
        self.record = record if record is not None else _torch_record
        self.run = run if run is not None else _torch_run
        self.free_memory = free_memory
        self.margin = margin
        self.max_requests_per_round = max_requests_per_round
        self.keys = {}
        self.queue = collections.deque()
        self.inflight = []
        self.reserved = 0
        self.lane_bytes = [0] * len(self.lanes)
        self.lane_cost = [0] * len(self.lanes)   # estimated device time queued on each lane and not yet finished
        self.rounds = []  # (round start, number of requests, clients, requests in flight before the round)
        self.failed = []  # requests whose batched call failed, handed back by the next poll

    def add_client(self, client, keys):
        self.keys[client] = keys

    def submit(self, req):
        if req.client not in self.keys:
            raise KeyError("unknown client %r" % (req.client,))
        self.queue.append(req)

    def admit(self):
        """Requests of the next round: the queue's head, in order, while the reservation fits the budget and the
        device's free memory.  With nothing in flight the head is always admitted (a request larger than the
        budget runs alone rather than never)."""
        taken, used = [], 0
        free = self.free_memory() if self.free_memory is not None else None
        while self.queue and len(taken) < self.max_requests_per_round:
            need = request_bytes(self.ctx, self.queue[0])
            busy = bool(taken) or bool(self.inflight)
            if busy and self.reserved + used + need > self.memory_budget:
                break
            if busy and free is not None and used + need + self.margin > free:
                break
            taken.append(self.queue.popleft())
            used += need
        return taken

    def poll(self):
        """Finished groups (their events complete): stamp their requests and release their memory.  Requests whose
        call failed come back at once, with .error set."""
        failed, self.failed = self.failed, []
        done, still = [], []
        for g in self.inflight:
            if g.event.query():
                done.append(g)
            else:
                still.append(g)
        if not done:
            return failed
        self.inflight = still
        now = self.clock()
        out = []
        for g in done:
            self.reserved -= g.bytes
            self.lane_bytes[g.lane] -= g.bytes
            self.lane_cost[g.lane] -= g.cost
            for r in g.reqs:
                r.done = now
            out += g.reqs
        return failed + out

    def launch(self, batch):
        """One round: the admitted requests grouped by client (clients in order of their first request), each group
        one batched call on the lane with the least estimated work queued, followed by an event on that lane's
        stream."""
        t0 = self.clock()
        by_client = collections.OrderedDict()
        for r in batch:
            r.start = t0
            by_client.setdefault(r.client, []).append(r)
        inflight_before = sum(len(g.reqs) for g in self.inflight)
        for client, reqs in by_client.items():
            nbytes = sum(request_bytes(self.ctx, r) for r in reqs)
            cost = sum(request_cost(r) for r in reqs)
            lane = min(range(len(self.lanes)), key=lambda i: (self.lane_cost[i], i))
            ctx = self.lanes[lane]
            try:
                outs = self.run(ctx, lambda: ctx.enc_matmul_batch(self.keys[client],
                                                                  [(r.op, r.a, r.b, r.c, r.t) for r in reqs]))
            except Exception as e:  # the library checks every request before any work: none of them ran
                for r in reqs:
                    r.error = e
                    r.lane = lane
                    r.done = self.clock()
                self.failed += reqs
                continue
            for r, o in zip(reqs, outs):
                r.result = o
                r.lane = lane
            self.inflight.append(_Group(reqs, self.record(ctx), nbytes, lane, cost))
            self.reserved += nbytes
            self.lane_bytes[lane] += nbytes
            self.lane_cost[lane] += cost
        self.rounds.append((t0, len(batch), len(by_client), inflight_before))

    def step(self):
        """Poll completions, then admit and launch what fits.  Returns the requests finished (or failed) since the
        last step."""
        finished = self.poll()
        batch = self.admit()
        if batch:
            self.launch(batch)
        return finished + self.poll_failed()

    def poll_failed(self):
        failed, self.failed = self.failed, []
        return failed

    def wait_one(self):
        """Block until the oldest group in flight is done (when there is nothing else to do)."""
        if self.inflight:
            self.inflight[0].event.synchronize()


def _torch_record(ctx):
    import torch
    ev = torch.cuda.Event()
    ev.record(ctx.stream)
    return ev


def _torch_run(ctx, fn):
    """fn with the lane's stream current; the lane first waits for the work queued on the default stream (which
    made the requests' inputs)."""
    import torch
    if ctx.stream != torch.cuda.default_stream(ctx.device):
        ctx.stream.wait_stream(torch.cuda.default_stream(ctx.device))
    with torch.cuda.stream(ctx.stream):
        return fn()


def concurrent_streams(count, candidates=32, spin_cycles=20_000_000):
    """`count` torch streams whose work runs side by side on the device.  Each candidate (from torch's stream pool)
    is used once, then kept if a small kernel on it finishes while a spin (about 10 ms) occupies every stream kept
    so far -- that is, if it did not land on the hardware queue of one of them.  RuntimeError if fewer qualify."""
    import torch
    dev = torch.cuda.current_device()
    probe = torch.zeros(256, device=dev)
    kept = []
    for _ in range(candidates):
        if len(kept) == count:
            break
        s = torch.cuda.Stream()
        if any(s == k for k in kept):
            continue
        with torch.cuda.stream(s):
            probe.add_(0.0)                   # first use: the runtime binds the stream to a hardware queue
        torch.cuda.synchronize()
        spins = []
        for k in kept:
            with torch.cuda.stream(k):
                torch.cuda._sleep(spin_cycles)
                ev = torch.cuda.Event()
                ev.record(k)
                spins.append(ev)
        with torch.cuda.stream(s):
            probe.add_(0.0)
            ev = torch.cuda.Event()
            ev.record(s)
        ev.synchronize()
        alone = all(not e.query() for e in spins)
        torch.cuda.synchronize()
        if alone:
            kept.append(s)
    if len(kept) < count:
        raise RuntimeError("only %d of %d streams run concurrently" % (len(kept), count))
    return kept


def poisson_arrivals(rng, rate, count, start=0.0):
    """`count` arrival times of a Poisson process of `rate` per second."""
    gaps = rng.exponential(1.0 / rate, size=count)
    out, t = [], start
    for g in gaps:
        t += float(g)
        out.append(t)
    return out


def serve(server, requests, clock=time.perf_counter, sleep=time.sleep, idle=2e-4):
    """Replay `requests` (their .arrival times, seconds from now) through `server`; returns them, finished.  When a
    step neither finishes nor admits anything, the loop waits `idle` seconds (or until the next arrival, if
    sooner) before polling again; with nothing in flight it sleeps until the next arrival."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    t_begin = clock()
    for r in pending:
        r.arrival += t_begin
    finished = []
    while pending or server.queue or server.inflight or server.failed:
        now = clock()
        while pending and pending[0].arrival <= now:
            server.submit(pending.popleft())
        queued = len(server.queue)
        done = server.step()
        finished += done
        if done or len(server.queue) < queued:
            continue
        if server.inflight:
            nxt = pending[0].arrival - clock() if pending else idle
            sleep(max(0.0, min(idle, nxt)))
        elif pending:
            sleep(max(0.0, pending[0].arrival - clock()))
    return finished


def latency_summary(finished, offered_rate):
    """p50 / p99 / max latency and the served rate of the requests that succeeded; failures are counted apart."""
    errors = sum(1 for r in finished if r.error is not None)
    finished = [r for r in finished if r.error is None]
    lat = sorted(r.latency for r in finished)
    span = max(r.done for r in finished) - min(r.arrival for r in finished)

    def pct(p):
        return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

    return dict(requests=len(finished), errors=errors, offered_per_s=offered_rate,
                served_per_s=round(len(finished) / span, 2),
                latency_ms_p50=round(1e3 * pct(50), 2), latency_ms_p99=round(1e3 * pct(99), 2),
                latency_ms_max=round(1e3 * lat[-1], 2))
