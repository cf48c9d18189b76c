"""GPU parity of the Goldbach check over a sieve table (include/sieve.h:
sieve_goldbach) against the CPU oracle (oracle_goldbach), element by element:
the least q of every even number and the per-segment maximum, its first argument
and the failures.  The oracle works on its own table (oracle_sieve), the GPU on the
table the HIP sieve wrote."""
import math
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_util import say, first_diff

pytestmark = pytest.mark.gpu


def gpu_goldbach(l, f, n, B, Q, per_number=True):
    import torch
    from paper_1111_3297_amd import api
    ctx = api.Context()
    pr = api.Primes(max(B, Q))
    S, c = api.alloc(l, n)
    ctx.sieve(l, f, n, B, S, c, primes=pr)
    maxq, argk, fails, minq = ctx.goldbach(pr, l, f, n, S, Q, per_number=per_number)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    h = lambda t: None if t is None else t.cpu().numpy()
    return S.cpu().numpy().view(np.uint32), h(minq), h(maxq).view(np.uint32), h(argk).view(np.uint64), \
        h(fails).view(np.uint32)


def check(l, f, n, B, Q):
    say("goldbach l=%d f=%d n=%d B=%d Q=%d" % (l, f, n, B, Q))
    S, minq, maxq, argk, fails = gpu_goldbach(l, f, n, B, Q)
    So, _ = O.sieve(l, f, n, B)
    assert first_diff(S, So) is None
    m, mx, ak, fl = O.goldbach(l, f, n, So, Q)
    d = np.flatnonzero(minq.view(np.uint32) != m)
    assert d.size == 0, ("minq", int(d[0]), int(minq[d[0]]), int(m[d[0]]), d.size)
    assert np.array_equal(maxq, mx) and np.array_equal(argk, ak) and np.array_equal(fails, fl)
    return m, mx, ak, fl


def test_goldbach_records_to_2_22():
    # 1 .. 2^22: the published records come out of the GPU as well (through the oracle)
    m, mx, ak, fl = check(15, 0, 64, 2048, 2048)
    assert int(mx.max()) == 751 and int(2 + 2 * ak[int(np.argmax(mx))]) == 3807404


@pytest.mark.parametrize("case", [
    (5, 0, 40, 100, 97),            # one word per segment: per-lane atomics, failures near the start
    (7, 3, 50, 1000, 1000),
    (12, 0, 9, 4096, 1621),         # exactly the 256 register-resident primes
    (12, 5, 9, 4096, 1619),         # 255 primes: the general loop only
    (12, 11, 9, 4096, 1627),        # 257 primes: one from the table
    (12, 3, 9, 4096, 727),
    (13, (10**9) >> 14, 5, 0, 13),  # Q = 13: failures everywhere; workgroup reduction
    (14, (10**9) >> 15, 3, 0, 40000),
    (16, (10**12) >> 17, 8, 0, 1 << 16),
    (20, (10**15) >> 21, 2, 0, 5000),
    (11, 1, 3, 300, 5000),          # partial table (B < isqrt(v)): zeros are rough numbers
])
def test_goldbach_cases(case):
    l, f, n, B, Q = case
    if B == 0:
        B = math.isqrt(O.interval(l, f, n)[1])
    check(l, f, n, B, Q)


@pytest.mark.parametrize("case", [
    (5, 0, 40, 100, 97),
    (12, 0, 9, 4096, 1621),
    (12, 11, 9, 4096, 1627),
    (13, (10**9) >> 14, 5, 0, 13),
    (14, (10**9) >> 15, 3, 0, 40000),
    (16, (10**12) >> 17, 8, 0, 1 << 16),
    (20, (10**15) >> 21, 2, 0, 5000),
    (15, 0, 64, 2048, 2048),
    (11, 1, 3, 300, 5000),
])
def test_goldbach_segment_outputs_only(case):
    # the kernel without per-number output (the benchmarked one): per-segment
    # maximum, first argument and failures against the oracle's
    l, f, n, B, Q = case
    if B == 0:
        B = math.isqrt(O.interval(l, f, n)[1])
    say("goldbach segments l=%d f=%d n=%d B=%d Q=%d" % (l, f, n, B, Q))
    S, _, maxq, argk, fails = gpu_goldbach(l, f, n, B, Q, per_number=False)
    So, _ = O.sieve(l, f, n, B)                 # the oracle's own table
    assert first_diff(S, So) is None
    _, mx, ak, fl = O.goldbach(l, f, n, So, Q, per_number=False)
    assert np.array_equal(maxq, mx) and np.array_equal(argk, ak) and np.array_equal(fails, fl)


def test_goldbach_full_size_sampled_segments():
    # the 2^33-number table at 1e12 (B = isqrt(v)), Q = 2^16, segment outputs only;
    # sampled segments recomputed by the oracle on a two-segment table that starts one
    # segment earlier (every q <= 2^16 reaches back less than one 2^20-bit segment)
    from paper_1111_3297_amd import workloads
    l, f, n, B = workloads.plain_configs()["interval_1e12"]
    Q = 1 << 16
    S, _, maxq, argk, fails = gpu_goldbach(l, f, n, B, Q, per_number=False)
    rng = random.Random(7)
    for t in [0, 1, 2047, 4095] + rng.sample(range(2, 4095), 4):
        say("sampled segment", t)
        if t == 0:
            So, _ = O.sieve(l, f, 1, B)
            _, mx, ak, fl = O.goldbach(l, f, 1, So, Q, per_number=False)
            got = (int(mx[0]), int(ak[0]), int(fl[0]))
        else:
            So, _ = O.sieve(l, f + t - 1, 2, B)
            _, mx, ak, fl = O.goldbach(l, f + t - 1, 2, So, Q, per_number=False)
            got = (int(mx[1]), int(ak[1]) + ((t - 1) << l), int(fl[1]))
        assert (int(maxq[t]), int(argk[t]), int(fails[t])) == got, t
    # only numbers below u + q for every q can fail: the first segment's first few
    assert int(fails[1:].sum()) == 0
