"""A request loop for encrypted matrix products on one GPU.

Clients submit DiagABT / DiagATB requests on ciphertexts already in device memory (block-encoded matrices made
with their own keys).  The server keeps every client's evaluation keys resident and serves the queue with
continuous batching: each round takes the queued requests in arrival order while their device-memory estimate fits
the budget (admission by memory), runs them as one batched call per client (`Context.enc_matmul_batch`, where
requests that share a shape class run in lockstep), waits for the device once, and stamps the completion time of
every request of the round.  A request's result is the same ciphertext it would get alone: the batched call is
bit-identical to single calls.
"""
import collections
import time


class Request:
    """One product: op "abt" (t A Bbar^T) or "atb" (t Abar^T B) on the client's matrices."""

    __slots__ = ("rid", "client", "op", "a", "b", "c", "t", "arrival", "start", "done", "result")

    def __init__(self, rid, client, op, a, b, c, t=1.0, arrival=0.0):
        if op not in ("abt", "atb"):
            raise ValueError("op must be 'abt' or 'atb'")
        self.rid, self.client, self.op, self.a, self.b, self.c, self.t = rid, client, op, a, b, c, t
        self.arrival = arrival
        self.start = self.done = None
        self.result = None

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


def request_bytes(ctx, req):
    """Device memory a request holds while it runs, bounded from above: its c/2 products per block pair (the
    Mult outputs, the tensor parts and the key-switch buffers of one launch group), plus its result."""
    half = req.c // 2
    if req.op == "abt":
        pairs = req.a.n_rb * req.a.n_cb
        level = min(req.a.level, req.b.level)
        out_blocks = req.a.n_rb
    else:
        pairs = req.b.n_rb * req.b.n_cb
        level = max(req.a.level, req.b.level)
        out_blocks = req.b.n_cb
    ct = ctx.ct_words(level) * 8
    return ct * (3 * half * pairs + out_blocks) + 40 * ct


class Server:
    """Continuous batching over a FIFO queue, with per-client keys and a device-memory admission budget."""

    def __init__(self, ctx, memory_budget, clock=time.perf_counter, sync=None, max_requests_per_round=256):
        self.ctx = ctx
        self.memory_budget = memory_budget
        self.clock = clock
        self.sync = sync
        self.max_requests_per_round = max_requests_per_round
        self.keys = {}
        self.queue = collections.deque()
        self.rounds = []  # (round start, number of requests, clients)

    def add_client(self, client, keys):
        self.keys[client] = keys

    def submit(self, req):
        if req.client not in self.keys:
            raise KeyError("unknown client %r" % (req.client,))
        self.queue.append(req)

    def admit(self):
        """Requests of the next round: the queue's head, in order, while the memory estimate fits.  The head is
        always admitted (a request larger than the budget runs alone rather than never)."""
        taken, used = [], 0
        while self.queue and len(taken) < self.max_requests_per_round:
            need = request_bytes(self.ctx, self.queue[0])
            if taken and used + need > self.memory_budget:
                break
            taken.append(self.queue.popleft())
            used += need
        return taken

    def step(self):
        """One round: admit, run one batched call per client (clients in order of their first queued request),
        wait for the device, stamp completions.  Returns the finished requests."""
        batch = self.admit()
        if not batch:
            return []
        t0 = self.clock()
        by_client = collections.OrderedDict()
        for r in batch:
            r.start = t0
            by_client.setdefault(r.client, []).append(r)
        for client, reqs in by_client.items():
            outs = self.ctx.enc_matmul_batch(self.keys[client], [(r.op, r.a, r.b, r.c, r.t) for r in reqs])
            for r, o in zip(reqs, outs):
                r.result = o
        if self.sync is not None:
            self.sync()
        t1 = self.clock()
        for r in batch:
            r.done = t1
        self.rounds.append((t0, len(batch), len(by_client)))
        return batch


def poisson_arrivals(rng, rate, count, start=0.0):
    """`count` arrival times of a Poisson process of `rate` per second."""
    gaps = rng.exponential(1.0 / rate, size=count)
    out, t = [], start
    for g in gaps:
        t += float(g)
        out.append(t)
    return out


def serve(server, requests, clock=time.perf_counter, sleep=time.sleep):
    """Replay `requests` (their .arrival times, seconds from now) through `server`; returns them, finished."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    t_begin = clock()
    for r in pending:
        r.arrival += t_begin
    finished = []
    while pending or server.queue:
        now = clock()
        while pending and pending[0].arrival <= now:
            server.submit(pending.popleft())
        if not server.queue:
            sleep(max(0.0, pending[0].arrival - clock()))
            continue
        finished += server.step()
    return finished


def latency_summary(finished, offered_rate):
    lat = sorted(r.latency for r in finished)
    span = max(r.done for r in finished) - min(r.arrival for r in finished)

    def pct(p):
        return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]

    return dict(requests=len(finished), offered_per_s=offered_rate, served_per_s=round(len(finished) / span, 2),
                latency_ms_p50=round(1e3 * pct(50), 2), latency_ms_p99=round(1e3 * pct(99), 2),
                latency_ms_max=round(1e3 * lat[-1], 2))
