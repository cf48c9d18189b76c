"""GPU parity of the batched persistent launch (include/sieve.h: sieve_batch).

Every request's table and counts in a batch must equal the CPU oracle's, and the
same request sieved alone (sieve_init) -- bit for bit, whatever the tile size the
batch runs with."""
import hashlib
import json
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_util import say, first_diff

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def run_batch(primes, l, reqs, tune=None):
    import torch
    from paper_1111_3297_amd import api
    ctx = api.Context()
    outs = []
    for (f, n, B) in reqs:
        S, c = api.alloc(l, n)
        S.fill_(-1)
        c.fill_(-1)
        outs.append((f, n, B, S, c))
    ctx.batch(primes, l, outs, tune=tune)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    return [(f, n, B, S.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32)) for (f, n, B, S, c) in outs]


def small_requests(seed, count, l):
    rng = random.Random(seed)
    reqs = []
    for _ in range(count):
        n = rng.randint(1, 4)
        e = rng.choice([0, 3, 6, 9, 11, 12, 13, 14])
        f = ((10**e) >> (l + 1)) + rng.randint(0, 9) if e else rng.randint(0, 3)
        u, v = O.interval(l, f, n)
        r = math.isqrt(v)
        B = rng.choice([r, r, max(3, r // 5), min(r, 13), min(r, 7)])
        reqs.append((f, n, max(3, B)))
    return reqs


@pytest.mark.parametrize("tune", [None, {"tile_log2": 17}, {"tile_log2": 18, "medium_log2": 15},
                                  {"tile_log2": 19, "medium_log2": 20, "wheel_log2": 12},
                                  {"tile_log2": 20, "medium_log2": 17, "bin_log2": 16}])
def test_batch_matches_oracle(tune):
    from paper_1111_3297_amd import api
    l = 20
    reqs = small_requests(7 if tune is None else 11, 10, l)
    Bmax = max(B for (_, _, B) in reqs)
    say("batch", tune, reqs)
    pr = api.Primes(Bmax)
    for (f, n, B, S, c) in run_batch(pr, l, reqs, tune):
        So, co = O.sieve(l, f, n, B)
        assert first_diff(S, So) is None, (f, n, B, tune, first_diff(S, So))
        assert np.array_equal(c, co), (f, n, B, tune)


def test_batch_small_segments_and_tiny_bounds():
    from paper_1111_3297_amd import api
    l = 12
    reqs = [(0, 5, 3), (0, 64, 2048), (7, 3, 13), ((10**9) >> 13, 40, 40000), ((10**12) >> 13, 17, 10**6)]
    pr = api.Primes(10**6)
    for tune in (None, {"tile_log2": 15, "medium_log2": 13, "bins_log2": 8}):
        say("batch l=12", tune)
        for (f, n, B, S, c) in run_batch(pr, l, reqs, tune):
            So, co = O.sieve(l, f, n, B)
            assert first_diff(S, So) is None, (f, n, B, tune)
            assert np.array_equal(c, co), (f, n, B, tune)


def test_batch_alone_vs_mix():
    # a request's result does not depend on the other requests of its batch
    import torch
    from paper_1111_3297_amd import api
    l = 20
    reqs = small_requests(99, 12, l)
    pr = api.Primes(max(B for (_, _, B) in reqs))
    mixed = run_batch(pr, l, reqs)
    for k in (0, 5, 11):
        f, n, B = reqs[k]
        S, c = api.alloc(l, n)
        api.sieve_init(l, f, n, B, S, c)
        torch.cuda.synchronize()
        assert np.array_equal(S.cpu().numpy().view(np.uint32), mixed[k][3])
        assert np.array_equal(c.cpu().numpy().view(np.uint32), mixed[k][4])
        alone = run_batch(pr, l, [reqs[k]])[0]
        assert np.array_equal(alone[3], mixed[k][3]) and np.array_equal(alone[4], mixed[k][4])


def test_batch_full_workload_against_oracle_golden():
    from paper_1111_3297_amd import api
    path = os.path.join(HERE, "golden", "batch_1234.json")
    if not os.path.exists(path):
        pytest.skip("golden file batch_1234 not generated")
    g = json.load(open(path))
    reqs = [(r["f"], r["n"], r["B"]) for r in g["requests"]]
    say("full batch", len(reqs), "requests")
    pr = api.Primes(max(B for (_, _, B) in reqs))
    res = run_batch(pr, g["l"], reqs)
    for (f, n, B, S, c), r in zip(res, g["requests"]):
        assert int(c.astype(np.int64).sum()) == r["total"], (f, n)
        assert hashlib.sha256(c.astype("<u4").tobytes()).hexdigest() == r["counts_sha256"], (f, n)
        assert hashlib.sha256(S.tobytes()).hexdigest() == r["S_sha256"], (f, n)
