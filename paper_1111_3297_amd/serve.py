"""Serving loop: continuous batching of interval requests over the batched launch.

A request is an interval of Section 1.2.1 at segment size 2^l, (f, n), sieved with
B = isqrt(v) (or a given bound).  The server replays an open-loop arrival
schedule, admits waiting requests first come first served as long as an in-flight
slot is free and the device memory budget allows (measured use plus an upper bound
of what the group adds: table, counts and the library's planned scratch), launches
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


# Allocator rounding that an upper bound of the device memory a request adds must
# cover, on top of the exact sizes: PyTorch's caching allocator takes a block of
# 2 MiB for a request of at most 1 MiB, 20 MiB below 10 MiB and whole 2 MiB units
# above; a library scratch buffer may end in a partly used 2 MiB page.
TORCH_SMALL, TORCH_MID, TORCH_UNIT = 2 << 20, 20 << 20, 2 << 20
LIB_BUFFERS, LIB_PAGE = 24, 2 << 20


def torch_block_bytes(nbytes):
    """Device bytes PyTorch's caching allocator may take for one tensor of nbytes."""
    if nbytes <= (1 << 20):
        return TORCH_SMALL
    if nbytes < (10 << 20):
        return TORCH_MID
    return -(-nbytes // TORCH_UNIT) * TORCH_UNIT


def request_bytes_bound(l, n, scratch):
    """Upper bound of the device bytes admitting a request adds: its table and counts
    as PyTorch allocates them, plus the library's planned scratch and a page of
    rounding for each of its buffers."""
    return torch_block_bytes((n << l) // 8) + torch_block_bytes(4 * n) + scratch + LIB_BUFFERS * LIB_PAGE


class GpuExecutor:
    """Runs groups of requests with sieve_batch, one context and stream per slot.
    With single_plain, a group of one runs as the plain per-interval call (less
    fixed cost), and so do, in groups of at most split_max requests, those with
    sparse large primes (sparse_plain), one after the other on the slot's stream
    before the batch of the rest: that shortens a heavy request's latency, while
    the large groups of a backlog keep their heavy requests in the batch, which
    serves the stream faster."""

    def __init__(self, primes, l, slots=3, tune=None, keep_outputs=False, single_plain=True, split_max=4):
        import torch
        from . import api
        self.torch = torch
        self.api = api
        self.primes = primes
        self.l = l
        self.tune = tune
        self.keep = keep_outputs
        self.single_plain = single_plain
        self.split_max = split_max
        self.slots = [{"ctx": api.Context(), "stream": torch.cuda.Stream(), "busy": False} for _ in range(slots)]
        self._cost = {}
        torch.cuda.synchronize()
        self._free0 = torch.cuda.mem_get_info()[0]   # free device memory before any request

    def free_slots(self):
        return sum(1 for s in self.slots if not s["busy"])

    def request_bytes(self, r):
        """Upper bound of the device bytes admitting r can add: its table and counts
        plus the scratch a fresh context would need for it (the planning pass of the
        library, for the batched and, when used, the plain call), with the
        allocators' rounding (request_bytes_bound)."""
        key = (r.f, r.n, r.B)
        c = self._cost.get(key)
        if c is None:
            ctx = self.slots[0]["ctx"]
            sc = ctx.batch_scratch_bytes(self.primes, self.l, [(r.f, r.n, r.B)], tune=self.tune)
            if self.single_plain:
                sc = max(sc, ctx.sieve_scratch_bytes(self.l, r.f, r.n, r.B, tune=self.tune, primes=self.primes))
            c = request_bytes_bound(self.l, r.n, sc)
            self._cost[key] = c
        return c

    def request_cost_ms(self, r):
        """Rough device time of r alone (a fit of measured plain calls on this device):
        launch overhead, tiles, and for bounds in the bucket range the per-prime work of
        the offsets and the bucket fill, which dominates heavy requests."""
        cost = 0.03 + 2e-4 * (r.n << self.l >> 20)
        if r.B >= (1 << 20):
            cost += 0.1 + 1.0e-8 * r.B / math.log(r.B)
        return cost

    def fixed_bytes(self):
        """Device bytes held whatever is admitted: the shared prime table."""
        return self.primes.nbytes()

    def device_bytes(self):
        """Device bytes in use now: the prime table plus what the device's free memory
        has dropped by since the executor was made (the slot contexts' scratch and the
        outputs of requests in flight, at the allocators' real granularity)."""
        return self.primes.nbytes() + max(0, self._free0 - self.torch.cuda.mem_get_info()[0])

    def trim_idle(self):
        """Free the scratch of idle slots and PyTorch's cached blocks."""
        for s in self.slots:
            if not s["busy"]:
                s["ctx"].trim()
        self.torch.cuda.empty_cache()

    def sparse_plain(self, n, B):
        """Whether a request has sparse large primes (p at least its table length of
        n 2^l bits, above the default medium bound 2^20): the plain call takes them
        on a path of their own, which batches do not have."""
        nb = n << self.l
        return nb > (1 << 20) and B >= min(nb, 1 << 31)

    def _launch(self, slot, outs):
        ctx, st = slot["ctx"], slot["stream"]
        if self.single_plain and len(outs) <= self.split_max:
            # a group of one, and a small group's requests with sparse large primes,
            # as plain calls
            one = len(outs) == 1
            for (f, n, B, S, c) in outs:
                if one or self.sparse_plain(n, B):
                    ctx.sieve(self.l, f, n, B, S, c, tune=self.tune, stream=st, primes=self.primes)
            outs = [o for o in outs if not (one or self.sparse_plain(o[1], o[2]))]
        if len(outs) == 1 and self.single_plain:
            f, n, B, S, c = outs[0]
            ctx.sieve(self.l, f, n, B, S, c, tune=self.tune, stream=st, primes=self.primes)
        elif outs:
            ctx.batch(self.primes, self.l, outs, tune=self.tune, stream=st)

    def submit(self, reqs):
        torch = self.torch
        slot = next(s for s in self.slots if not s["busy"])
        slot["busy"] = True
        with torch.cuda.stream(slot["stream"]):
            outs = []
            for r in reqs:
                S, c = self.api.alloc(self.l, r.n)
                outs.append((r.f, r.n, r.B, S, c))
            self._launch(slot, outs)
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
        super().__init__(primes, l, slots=1, tune=tune, keep_outputs=keep_outputs, single_plain=True)

    def request_bytes(self, r):
        key = (r.f, r.n, r.B)
        c = self._cost.get(key)
        if c is None:
            ctx = self.slots[0]["ctx"]
            c = request_bytes_bound(self.l, r.n, ctx.sieve_scratch_bytes(self.l, r.f, r.n, r.B, tune=self.tune,
                                                                         primes=self.primes))
            self._cost[key] = c
        return c

    def _launch(self, slot, outs):
        for f, n, B, S, c in outs:
            slot["ctx"].sieve(self.l, f, n, B, S, c, tune=self.tune, stream=slot["stream"], primes=self.primes)


class Server:
    """Open-loop replay with device-memory budget admission and continuous batching.

    Admission measures the device memory in use (executor.device_bytes(): the prime
    table, the slot contexts' scratch and PyTorch's allocator) and admits the next
    waiting request into the group being formed while that, plus the upper bounds of
    the group's requests (executor.request_bytes), stays within the budget and the
    group's estimated device time (executor.request_cost_ms) within group_ms, or
    within the waiting work's share per free slot when that is larger (a request
    heavier than the cap forms a group of its own).  A request that does not
    fit while idle slots hold scratch frees that scratch first."""

    def __init__(self, executor, l=20, budget_bytes=64 << 30, max_group=64, group_ms=0.5, poll_s=20e-6, clock=None,
                 sleep=None, progress=None, progress_s=10.0):
        self.ex = executor
        self.l = l
        self.budget = budget_bytes
        self.max_group = max_group
        self.group_ms = group_ms
        self.poll_s = poll_s
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.progress = progress
        self.progress_s = progress_s
        self.peak_bytes = 0
        self.trims = 0

    def run(self, requests):
        """requests: Requests sorted by arrival (seconds from start).  Returns
        (results by rid, stats)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        fixed = self.ex.fixed_bytes()
        for r in reqs:
            if fixed + self.ex.request_bytes(r) > self.budget:
                raise ValueError("request %s alone exceeds the device memory budget" % (r.rid,))
        pending = collections.deque()
        pending_ms = 0.0            # estimated device time of the waiting requests
        inflight = []
        results, lat = {}, {}
        i = 0
        t0 = self.clock()
        last_done = 0.0
        next_report = self.progress_s
        while i < len(reqs) or pending or inflight:
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                pending.append(reqs[i])
                pending_ms += self.ex.request_cost_ms(reqs[i])
                i += 1
            if self.progress and now >= next_report:
                self.progress(now, len(results), len(reqs))
                next_report += self.progress_s
            # retire finished groups
            still = []
            for h in inflight:
                if self.ex.done(h):
                    out = self.ex.finish(h)
                    tdone = self.clock() - t0
                    last_done = tdone
                    for r in h["reqs"]:
                        results[r.rid] = out[r.rid]
                        lat[r.rid] = tdone - r.arrival
                else:
                    still.append(h)
            inflight = still
            # admit: first come first served, as many as fit the budget
            trimmed = False
            while pending and self.ex.free_slots() > 0:
                used = self.ex.device_bytes()
                # under a backlog the free slots share the waiting work, so groups
                # grow with it (batching pays most when the device is saturated)
                cap_ms = max(self.group_ms, pending_ms / max(1, self.ex.free_slots()))
                group, gbytes, gms = [], 0, 0.0
                while pending and len(group) < self.max_group:
                    cb = self.ex.request_bytes(pending[0])
                    cm = self.ex.request_cost_ms(pending[0])
                    if used + gbytes + cb > self.budget:
                        break
                    # a group holds about group_ms of device work, so that light
                    # requests do not wait behind a heavy one of the same group
                    if group and gms + cm > cap_ms:
                        break
                    group.append(pending.popleft())
                    gbytes += cb
                    gms += cm
                    pending_ms -= cm
                if not group:
                    if not trimmed:
                        self.ex.trim_idle()
                        self.trims += 1
                        trimmed = True
                        continue
                    break
                h = self.ex.submit(group)
                self.peak_bytes = max(self.peak_bytes, self.ex.device_bytes())
                inflight.append(h)
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
                 "budget_bytes": self.budget, "trims": self.trims}
        return results, stats


def serving_requests(l=20, seed=99, rate=200.0, seconds=60.0, limit_s=None, speedup=1.0):
    """The seeded Poisson stream of paper_1111_3297_amd.workloads as Requests with
    B = isqrt(v); limit_s keeps only arrivals before that time (of the original
    stream); speedup divides every arrival time (the same requests offered faster)."""
    from . import workloads
    out = []
    for k, (t, f21, n21, kind) in enumerate(workloads.serving_stream(seed, rate, seconds)):
        if limit_s is not None and t >= limit_s:
            break
        f, n = f21 << (20 - l), n21 << (20 - l)
        u, v = workloads.interval(l, f, n)
        out.append(Request(k, t / speedup, f, n, math.isqrt(v)))
    return out
