"""Serving loop: continuous batching of interval requests over the batched launch.

A request is an interval of Section 1.2.1 at segment size 2^l, (f, n), sieved with
B = isqrt(v) (or a given bound).  The server replays an open-loop arrival
schedule, admits waiting requests first come first served as long as an in-flight
slot is free and the HBM budget (table + counts + batch scratch) allows, launches
each admitted group as one sieve_batch (a group of one as the plain per-interval
call, which costs less) on that slot's own context and stream, and
retires slots by polling their completion events.  Requests that arrive while
others are on the GPU join the next group as soon as a slot and memory free up,
and groups on different slots overlap on the device.  Latency of a request is the
host time its counts reach host memory minus its scheduled arrival.

The GPU work is done by an executor; GpuExecutor drives libsieve.so.  Tests use a
CPU executor with the same interface to check admission and accounting.
"""
import collections
import math
import time

Request = collections.namedtuple("Request", "rid arrival f n B")


def request_bytes(l, n):
    """Device bytes a request's outputs occupy: the table and its counts."""
    return (n << l) // 8 + 4 * n


class GpuExecutor:
    """Runs groups of requests with sieve_batch, one context and stream per slot."""

    def __init__(self, primes, l, slots=3, tune=None, keep_outputs=False):
        import torch
        from . import api
        self.torch = torch
        self.api = api
        self.primes = primes
        self.l = l
        self.tune = tune
        self.keep = keep_outputs
        self.slots = [{"ctx": api.Context(), "stream": torch.cuda.Stream(), "busy": False} for _ in range(slots)]

    def free_slots(self):
        return sum(1 for s in self.slots if not s["busy"])

    def scratch_bytes(self, reqs):
        ctx = self.slots[0]["ctx"]
        return ctx.batch_scratch_bytes(self.primes, self.l, [(r.f, r.n, r.B) for r in reqs], tune=self.tune)

    def submit(self, reqs):
        torch = self.torch
        slot = next(s for s in self.slots if not s["busy"])
        slot["busy"] = True
        with torch.cuda.stream(slot["stream"]):
            outs = []
            for r in reqs:
                S, c = self.api.alloc(self.l, r.n)
                outs.append((r.f, r.n, r.B, S, c))
            if len(outs) == 1:
                # a group of one (light load): the plain per-interval call has less
                # fixed cost than a batch of one, with the same result
                f, n, B, S, c = outs[0]
                slot["ctx"].sieve(self.l, f, n, B, S, c, tune=self.tune, stream=slot["stream"], primes=self.primes)
            else:
                slot["ctx"].batch(self.primes, self.l, outs, tune=self.tune, stream=slot["stream"])
            host_counts = [torch.empty(r.n, dtype=torch.int32, pin_memory=True) for r in reqs]
            for hc, o in zip(host_counts, outs):
                hc.copy_(o[4], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(slot["stream"])
        return {"slot": slot, "reqs": reqs, "outs": outs, "host_counts": host_counts, "event": ev}

    def done(self, h):
        return h["event"].query()

    def finish(self, h):
        h["event"].synchronize()
        h["slot"]["ctx"].check_device_errors()
        h["slot"]["busy"] = False
        res = {}
        for r, hc, o in zip(h["reqs"], h["host_counts"], h["outs"]):
            res[r.rid] = {"counts": hc.numpy().view("uint32").copy()}
            if self.keep:
                res[r.rid]["S"] = o[3]
        h["outs"] = None
        return res


class PlainExecutor(GpuExecutor):
    """First come first served with the plain per-interval sieve: one request at a
    time on one stream, shared prime table (the baseline for the batched server)."""

    def __init__(self, primes, l, tune=None, keep_outputs=False):
        super().__init__(primes, l, slots=1, tune=tune, keep_outputs=keep_outputs)

    def scratch_bytes(self, reqs):
        return super().scratch_bytes(reqs)

    def submit(self, reqs):
        torch = self.torch
        slot = self.slots[0]
        slot["busy"] = True
        with torch.cuda.stream(slot["stream"]):
            outs, host_counts = [], []
            for r in reqs:
                S, c = self.api.alloc(self.l, r.n)
                slot["ctx"].sieve(self.l, r.f, r.n, r.B, S, c, tune=self.tune, stream=slot["stream"],
                                  primes=self.primes)
                hc = torch.empty(r.n, dtype=torch.int32, pin_memory=True)
                hc.copy_(c, non_blocking=True)
                outs.append((r.f, r.n, r.B, S, c))
                host_counts.append(hc)
            ev = torch.cuda.Event()
            ev.record(slot["stream"])
        return {"slot": slot, "reqs": reqs, "outs": outs, "host_counts": host_counts, "event": ev}


class Server:
    """Open-loop replay with HBM-budget admission and continuous batching."""

    def __init__(self, executor, l=20, budget_bytes=64 << 30, max_group=64, poll_s=20e-6, clock=None, sleep=None):
        self.ex = executor
        self.l = l
        self.budget = budget_bytes
        self.max_group = max_group
        self.poll_s = poll_s
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.peak_bytes = 0
        self._cost = {}

    def cost_bytes(self, reqs):
        """Budget charge of a group: outputs plus batch scratch, summed per request
        (the scratch estimate is additive over requests)."""
        tot = 0
        for r in reqs:
            c = self._cost.get(r.rid)
            if c is None:
                c = request_bytes(self.l, r.n) + self.ex.scratch_bytes([r])
                self._cost[r.rid] = c
            tot += c
        return tot

    def run(self, requests):
        """requests: Requests sorted by arrival (seconds from start).  Returns
        (results by rid, stats)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            if self.cost_bytes([r]) > self.budget:
                raise ValueError("request %s alone exceeds the HBM budget" % (r.rid,))
        pending = collections.deque()
        inflight = []
        used = 0
        results, lat = {}, {}
        i = 0
        t0 = self.clock()
        first_launch = None
        last_done = 0.0
        while i < len(reqs) or pending or inflight:
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                pending.append(reqs[i])
                i += 1
            # retire finished groups
            still = []
            for h, nbytes in inflight:
                if self.ex.done(h):
                    out = self.ex.finish(h)
                    tdone = self.clock() - t0
                    last_done = tdone
                    for r in h["reqs"]:
                        results[r.rid] = out[r.rid]
                        lat[r.rid] = tdone - r.arrival
                    used -= nbytes
                else:
                    still.append((h, nbytes))
            inflight = still
            # admit: first come first served, as many as fit the budget
            while pending and self.ex.free_slots() > 0:
                group, gbytes = [], 0
                while pending and len(group) < self.max_group:
                    cb = self.cost_bytes([pending[0]])
                    if used + gbytes + cb > self.budget:
                        break
                    group.append(pending.popleft())
                    gbytes += cb
                if not group:
                    break
                h = self.ex.submit(group)
                if first_launch is None:
                    first_launch = self.clock() - t0
                used += gbytes
                self.peak_bytes = max(self.peak_bytes, used)
                inflight.append((h, gbytes))
            if not inflight and not pending and i < len(reqs):
                wait = reqs[i].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 0.002))
            elif inflight:
                self.sleep(self.poll_s)
        span = max(last_done, 1e-9)
        numbers = sum(r.n << (self.l + 1) for r in reqs)
        ls = sorted(lat.values())

        def pct(q):
            if not ls:
                return float("nan")
            return ls[min(len(ls) - 1, max(0, int(math.ceil(q * len(ls))) - 1))]

        stats = {"requests": len(reqs), "numbers": numbers, "span_s": span,
                 "numbers_per_s": numbers / span, "p50_ms": 1e3 * pct(0.50), "p99_ms": 1e3 * pct(0.99),
                 "max_ms": 1e3 * (ls[-1] if ls else float("nan")), "peak_bytes": self.peak_bytes,
                 "budget_bytes": self.budget}
        return results, stats


def serving_requests(l=20, seed=99, rate=200.0, seconds=60.0, limit_s=None):
    """The seeded Poisson stream of paper_1111_3297_amd.workloads as Requests with
    B = isqrt(v); limit_s keeps only arrivals before that time."""
    from . import workloads
    out = []
    for k, (t, f21, n21, kind) in enumerate(workloads.serving_stream(seed, rate, seconds)):
        if limit_s is not None and t >= limit_s:
            break
        f, n = f21 << (20 - l), n21 << (20 - l)
        u, v = workloads.interval(l, f, n)
        out.append(Request(k, t, f, n, math.isqrt(v)))
    return out
