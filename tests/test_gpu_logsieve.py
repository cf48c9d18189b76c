"""GPU parity of the log-add sieve (include/sieve.h: sieve_logsieve) against the
CPU oracle (oracle_logsieve), element by element: the byte sums, the candidate bit
table and the candidates per segment."""
import math
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_util import say, first_diff

pytestmark = pytest.mark.gpu


def gpu_logsieve(l, f, n, B, T, tune=None, sums=True):
    import torch
    from paper_1111_3297_amd import api
    ctx = api.Context()
    C, c = api.alloc(l, n)
    A = torch.empty(n << l, dtype=torch.uint8, device="cuda") if sums else None
    ctx.logsieve(l, f, n, B, T, C, c, A=A, tune=tune)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    return C.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32), None if A is None else A.cpu().numpy()


def check(l, f, n, B, T, tune=None):
    say("logsieve l=%d f=%d n=%d B=%d T=%d tune=%s" % (l, f, n, B, T, tune))
    C, c, A = gpu_logsieve(l, f, n, B, T, tune)
    Co, co, Ao = O.logsieve(l, f, n, B, T)
    d = np.flatnonzero(A != Ao)
    assert d.size == 0, ("sums", int(d[0]), int(A[d[0]]), int(Ao[d[0]]), d.size)
    assert first_diff(C, Co) is None, first_diff(C, Co)
    assert np.array_equal(c, co)


@pytest.mark.parametrize("case", [
    (10, 0, 8, 1000, 7),                 # from the number 1, primes counting themselves
    (5, 3, 40, 97, 5),                   # one word per segment
    (12, (10**9) >> 13, 16, 40000, 20),  # medium primes only
    (16, (10**9) >> 17, 6, 70000, 24),   # bucket path (primes >= 2^16)
    (20, (10**12) >> 21, 2, 10**6, 30),  # segments longer than tiles, ragged bucket bins
    (15, 7, 9, 3, 1),                    # B = 3
    (14, 100, 5, 5000, 0),               # T = 0: every bit set
    (14, 100, 5, 5000, 255),             # T = 255: none
])
def test_logsieve_cases(case):
    check(*case)


@pytest.mark.parametrize("B", [4, 5, 6, 7, 10, 11, 12, 13, 16, 17, 19])
def test_logsieve_small_prime_pattern_bounds(B):
    # the weights of 3..13 come from a periodic pattern holding only the primes up
    # to B; from the number 1 (the primes count themselves) and far from it
    check(10, 0, 4, B, 1)
    check(12, 15015 * 1000 + 77, 3, B, 2)


@pytest.mark.parametrize("tile", [14, 15, 16, 17])
def test_logsieve_tile_sizes(tile):
    check(17, (10**11) >> 18, 6, 300007, 25, tune={"tile_log2": tile})


@pytest.mark.parametrize("tune", [{"groups": 256}, {"tile_log2": 16, "ranges": 2, "groups": 2048},
                                  {"ranges": 1, "groups": 64}, {"ranges": 8}])
def test_logsieve_bucket_layouts(tune):
    check(18, (10**12) >> 19, 40, 2 * 10**6 + 11, 28, tune=tune)


def test_logsieve_multi_chunk_and_windows():
    # 2^28 positions: two chunks of 2^11 bins of 2^16 positions, B well past the tile
    check(20, (10**13) >> 21, 256, 3 * 10**6, 32, tune={"tile_log2": 16, "groups": 256})
    # 2^29 positions at the default tiles of 2^17: two chunks of 2^11 bins
    check(20, (10**13) >> 21, 512, 3 * 10**6, 32)


def test_logsieve_full_size_sampled_segments():
    # the 2^33-number interval at 1e12 with the primes below 2^20: candidate tables of
    # sampled segments against the oracle (a position's sum depends on its number only)
    from paper_1111_3297_amd import workloads
    l, f, n, _ = workloads.plain_configs()["interval_1e12"]
    B, T = 1 << 20, 30
    C, c, _ = gpu_logsieve(l, f, n, B, T, sums=False)
    w = 1 << (l - 5)
    for t in [0, 1, 2048, 4095] + random.Random(3).sample(range(2, 4095), 3):
        say("sampled segment", t)
        Co, co, _ = O.logsieve(l, f + t, 1, B, T, with_sums=False)
        assert first_diff(C[t * w:(t + 1) * w], Co) is None, t
        assert int(c[t]) == int(co[0]), t
