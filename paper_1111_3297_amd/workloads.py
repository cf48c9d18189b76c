"""Seeded synthetic inputs (interval requests).  No sieve arithmetic lives here:
these functions only draw interval parameters, which both the GPU path and the
CPU oracle then receive.

Interval parameters follow Section 1.2.1: (l, f, n) give u = f*2^(l+1)+1 and
v = (f+n)*2^(l+1).  Batched and served requests are quantised to whole 2^21-number
blocks (f21, n21 at l = 20), so that any tile size 2^17..2^20 bits divides them.
"""
import math

import numpy as np

Q = 1 << 21  # numbers per 2^20-bit block


def interval(l, f, n):
    return f * (1 << (l + 1)) + 1, (f + n) * (1 << (l + 1))


def plain_configs():
    """The single-interval workloads (l, f, n, B) used by tests and the benchmark."""
    f12 = (10**12 - 2**32) // 2**21
    u, v = interval(20, f12, 4096)
    return {
        "interval_2p22": (15, 0, 64, 2048),                 # sieves 1..2^22 with primes <= 2048
        "interval_1e12": (20, f12, 4096, math.isqrt(v)),     # 2^33 numbers centred at 1e12
        "interval_1e12_b6": (20, f12, 4096, 10**6),          # same interval, literal bound 10^6
        "interval_2p60": (20, 2**39 - 2048, 4096, 2**30),    # 2^33 numbers centred at 2^60
        # the serving stream's request of largest bound: 2^28 numbers near 9.1e18
        "serve_req6388": (20, 2171055560302, 128, 2133783848),
    }


def _quantise(c, w):
    n21 = max(1, int(round(w / Q)))
    f21 = max(0, int(c) // Q - n21 // 2)
    return f21, n21


def batch_requests(seed=1234, count=256):
    """256 requests: centres log-uniform in [1e6, 1e15], widths log-uniform in
    [2^20, 2^30] numbers, rounded to whole 2^21-number blocks.  Returns a list of
    (f21, n21) at l = 20."""
    rng = np.random.default_rng(seed)
    c = 10 ** rng.uniform(6, 15, count)
    w = 2 ** rng.uniform(20, 30, count)
    return [_quantise(ci, wi) for ci, wi in zip(c, w)]


def serving_stream(seed=99, rate=200.0, seconds=60.0):
    """Poisson arrivals (mean `rate` per second for `seconds`): 90% of requests as
    in batch_requests, 10% with centres log-uniform in [1e16, 2^62] and width
    2^28.  Returns a list of (arrival_s, f21, n21, kind)."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        if rng.random() < 0.9:
            c = 10 ** rng.uniform(6, 15)
            w = 2 ** rng.uniform(20, 30)
            kind = "A"
        else:
            c = math.exp(rng.uniform(math.log(1e16), math.log(2.0**62)))
            w = 2.0**28
            kind = "B"
        f21, n21 = _quantise(c, w)
        out.append((t, f21, n21, kind))
    return out
