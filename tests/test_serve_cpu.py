"""CPU tests of the serving scheduler (paper_1111_3297_amd/serve.py) with a fake
executor backed by the CPU oracle and a virtual clock: admission never exceeds
the byte budget, requests start first come first served, every request gets the
oracle's counts, and latency is measured from the scheduled arrival."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1111_3297_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Completes a group `service_s` seconds of virtual time after submission.  Each
    slot keeps the scratch of its largest group (as a library context keeps its
    grown buffers) until trim_idle frees it; device_bytes is that plus the outputs
    and scratch of the groups in flight."""

    def __init__(self, clock, l, slots=2, service_s=0.01, scratch=1000):
        self.clock, self.l, self.nslots, self.service_s, self.scratch = clock, l, slots, service_s, scratch
        self.order = []
        self.retained = [0] * slots
        self.busy = [None] * slots
        self.trims = 0

    def free_slots(self):
        return sum(1 for b in self.busy if b is None)

    def request_bytes(self, r):
        return serve.request_bytes(self.l, r.n) + self.scratch

    def fixed_bytes(self):
        return 0

    def request_cost_ms(self, r):
        return 0.0

    def device_bytes(self):
        out = sum(self.retained)
        for b in self.busy:
            if b is not None:
                out += sum(serve.request_bytes(self.l, r.n) for r in b["reqs"])
        return out

    def trim_idle(self):
        self.trims += 1
        for k, b in enumerate(self.busy):
            if b is None:
                self.retained[k] = 0

    def submit(self, reqs):
        k = self.busy.index(None)
        h = {"reqs": reqs, "t_done": self.clock.now() + self.service_s, "slot": k}
        self.busy[k] = h
        self.retained[k] = max(self.retained[k], self.scratch * len(reqs))
        self.order.extend(r.rid for r in reqs)
        return h

    def done(self, h):
        return self.clock.now() >= h["t_done"]

    def finish(self, h):
        self.busy[h["slot"]] = None
        out = {}
        for r in h["reqs"]:
            _, c = O.sieve(self.l, r.f, r.n, r.B)
            out[r.rid] = {"counts": c}
        return out


def make_requests(l, k, rate, seed=3):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for rid in range(k):
        t += rng.exponential(1.0 / rate)
        n = int(rng.integers(1, 4))
        f = int(rng.integers(0, 1 << 20))
        u, v = O.interval(l, f, n)
        out.append(serve.Request(rid, t, f, n, math.isqrt(v)))
    return out


def test_all_requests_served_with_oracle_counts_in_arrival_order():
    clock = FakeClock()
    l = 10
    ex = FakeExecutor(clock, l, slots=2, service_s=0.005)
    srv = serve.Server(ex, l=l, budget_bytes=1 << 30, clock=clock.now, sleep=clock.sleep)
    reqs = make_requests(l, 60, rate=500.0)
    res, st = srv.run(reqs)
    assert sorted(res) == [r.rid for r in reqs]
    assert ex.order == [r.rid for r in reqs]          # first come first served
    for r in reqs:
        _, c = O.sieve(l, r.f, r.n, r.B)
        assert np.array_equal(res[r.rid]["counts"], c)
    assert st["p50_ms"] >= 5.0 - 1e-6                  # at least the service time
    assert st["p99_ms"] >= st["p50_ms"]


def test_budget_is_never_exceeded():
    # retained scratch of idle slots counts against the budget and is freed when a
    # waiting request would not fit otherwise
    clock = FakeClock()
    l = 10
    ex = FakeExecutor(clock, l, slots=8, service_s=0.05, scratch=4000)
    per = serve.request_bytes(l, 3) + 4000
    budget = 5 * per
    seen = []
    orig = ex.device_bytes

    def spy():
        v = orig()
        seen.append(v)
        return v
    ex.device_bytes = spy
    srv = serve.Server(ex, l=l, budget_bytes=budget, clock=clock.now, sleep=clock.sleep)
    reqs = make_requests(l, 40, rate=2000.0, seed=5)
    res, st = srv.run(reqs)
    assert len(res) == 40
    assert st["peak_bytes"] <= budget
    assert max(seen) <= budget
    assert ex.trims > 0


def test_request_larger_than_budget_is_rejected():
    clock = FakeClock()
    l = 10
    ex = FakeExecutor(clock, l)
    srv = serve.Server(ex, l=l, budget_bytes=10, clock=clock.now, sleep=clock.sleep)
    with pytest.raises(ValueError):
        srv.run(make_requests(l, 2, rate=10.0))


def test_latency_counts_from_scheduled_arrival_when_slots_are_full():
    clock = FakeClock()
    l = 10
    ex = FakeExecutor(clock, l, slots=1, service_s=0.1)
    srv = serve.Server(ex, l=l, budget_bytes=1 << 30, max_group=1, clock=clock.now, sleep=clock.sleep)
    reqs = [serve.Request(k, 0.0, 5 + k, 1, 100) for k in range(3)]
    res, st = srv.run(reqs)
    # one slot, one request per group: completions at 0.1, 0.2, 0.3 s after arrival 0
    assert abs(st["max_ms"] - 300.0) < 1.0
    assert abs(st["p50_ms"] - 200.0) < 1.0


def test_request_bound_covers_allocator_rounding():
    # PyTorch's caching allocator: 2 MiB blocks up to 1 MiB, 20 MiB below 10 MiB,
    # whole 2 MiB units above; the bound adds a page per library buffer
    assert serve.torch_block_bytes(512) == 2 << 20
    assert serve.torch_block_bytes((1 << 20) + 1) == 20 << 20
    assert serve.torch_block_bytes(16 << 20) == 16 << 20
    assert serve.torch_block_bytes((16 << 20) + 1) == 18 << 20
    for l, n in [(10, 1), (20, 3), (20, 128), (16, 4096)]:
        exact = serve.request_bytes(l, n)
        b = serve.request_bytes_bound(l, n, 12345)
        assert b >= exact + 12345 + serve.LIB_BUFFERS * serve.LIB_PAGE


def test_sparse_plain_rule():
    # sparse large primes exist when the table is longer than the medium bound 2^20
    # and B reaches its length (capped at one 2^31-bit window)
    class E:
        l = 20
    sp = lambda n, B: serve.GpuExecutor.sparse_plain(E, n, B)
    assert not sp(1, 10**9)                 # 2^20 bits: every large prime is bucketed
    assert sp(128, 2**27) and not sp(128, 2**27 - 1)
    assert sp(4096, 2**31) and not sp(4096, 2**31 - 1)
