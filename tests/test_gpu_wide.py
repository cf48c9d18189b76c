"""GPU parity of intervals beyond 2^64 (include/sieve.h: sieve_wide) against the
CPU oracle's Definition 1 with a 128-bit start (oracle_sieve_wide), bit for bit.

Small bounds compare whole tables with the oracle directly; bounds at and above
2^32 (the primes of more than 32 bits, Section 5) compare per-segment counts and
the SHA-256 of the table with values the oracle wrote
(tests/golden/make_golden.py).  At the size the benchmark times, sampled bits are
checked against a Miller-Rabin test (B >= isqrt(v): zero bit <=> prime)."""
import json
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_util import say, sha256_words, first_diff

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def gpu_wide(l, f, n, B, ctx=None, tune=None):
    import torch
    from paper_1111_3297_amd import api
    S, c = api.alloc(l, n)
    ctx = ctx or api.Context()
    ctx.wide(l, f, n, B, S, c, tune=tune)
    torch.cuda.synchronize()
    ctx.check_device_errors()
    return S.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32)


def check_wide(l, f, n, B, ctx=None):
    say("wide case l=%d f=%d n=%d B=%d" % (l, f, n, B))
    S, c = gpu_wide(l, f, n, B, ctx)
    So, co = O.sieve_wide(l, f, n, B)
    assert first_diff(S, So) is None, ("table", l, f, n, B, first_diff(S, So))
    assert np.array_equal(c, co), ("counts", l, f, n, B)


@pytest.mark.parametrize("case", [
    (10, 2**54 + 777, 37, 65537),            # medium primes only
    (5, 2**58, 100, 1000003),                # u = 2^64 + 1, 32-bit segments
    (20, 2**80 + 3, 3, 2**24 + 7),           # large primes through the buckets
    (13, 2**114 - 1001, 1000, 3000017),      # v = 2^128 - 2^14, the largest end
    (15, 3 * 2**100 + 11, 64, 2048),
    (17, 2**64 - 5, 24, 10**6 + 3),          # f itself above 2^64
    (20, 2**43 + 7, 2049, 2**21 + 1),        # two launch windows
])
def test_wide_against_oracle(case):
    check_wide(*case)


def test_wide_context_reuse():
    # one context: a wide call between two ordinary ones leaves both right
    from paper_1111_3297_amd import api
    from tests.gpu_util import gpu_sieve
    ctx = api.Context()
    S, c = gpu_sieve(20, 474789, 8, 1002145, ctx=ctx)
    So, co = O.sieve(20, 474789, 8, 1002145)
    assert np.array_equal(S, So) and np.array_equal(c, co)
    check_wide(12, 2**60 + 99, 50, 200003, ctx=ctx)
    S, c = gpu_sieve(20, 474789, 8, 1002145, ctx=ctx)
    assert np.array_equal(S, So) and np.array_equal(c, co)


def test_wide_rejections():
    import torch
    from paper_1111_3297_amd import api, _lib
    S, c = api.alloc(12, 4)
    ctx = api.Context()
    bad = [
        ((12, 2**51 - 1, 4, 1000), "SIEVE_E_RANGE"),       # u = 2^64 - 2^13 + 1 < 2^64
        ((12, 2**115 - 4, 4, 1000), "SIEVE_E_RANGE"),      # v = 2^128
        ((12, 2**51, 4, 2**40 + 1), "SIEVE_E_BOUND"),
        ((12, 2**51, 4, 2), "SIEVE_E_BOUND"),
    ]
    for args, name in bad:
        with pytest.raises(_lib.SieveError) as e:
            ctx.wide(*args, S, c)
        assert name in str(e.value), (args, str(e.value))
    torch.cuda.synchronize()


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % name)
    with open(path) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name", ["wide_2p66", "wide_b32", "wide_top", "wide_u2p64", "wide_2p66_2g", "wide_2p68"])
def test_wide_against_oracle_golden(name):
    g = _golden(name)
    l, f, n, B = g["l"], int(g["f"]), g["n"], g["B"]
    say("wide golden %s l=%d f=%d n=%d B=%d" % (name, l, f, n, B))
    S, c = gpu_wide(l, f, n, B)
    assert [int(x) for x in c] == g["counts"], name
    assert sha256_words(S) == g["S_sha256"], name


@pytest.mark.parametrize("name,tune", [
    ("wide_2p66_2g", {"wide_list": 1}),             # every hit OR-ed in with atomics
    ("wide_2p66_2g", {"wide_slot_log2": 6}),        # 64-entry slots: most hits overflow to atomics
    ("wide_2p66_2g", {"wide_sort_hits": 30000}),    # sorting workgroups past 8192 hits: the rest by atomics
    ("wide_2p66", {"wide_list": 2}),                # a sparse slice listed and sorted all the same
    ("wide_2p68", {"wide_list": 2, "wide_slot_log2": 13, "wide_sort_hits": 16}),
])
def test_wide_hit_paths_against_oracle_golden(name, tune):
    # the ways a hit of a prime above 2^32 reaches the table, forced through the
    # wide_* tuning fields: each against the oracle's golden
    g = _golden(name)
    l, f, n, B = g["l"], int(g["f"]), g["n"], g["B"]
    say("wide golden %s l=%d f=%d n=%d B=%d tune=%s" % (name, l, f, n, B, tune))
    S, c = gpu_wide(l, f, n, B, tune=tune)
    assert [int(x) for x in c] == g["counts"], (name, tune)
    assert sha256_words(S) == g["S_sha256"], (name, tune)


def _is_probable_prime(N):
    # Miller-Rabin to the first twelve prime bases (deterministic below 3.1e23,
    # a probable-prime test above)
    if N < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if N % p == 0:
            return N == p
    d, s = N - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, N)
        if x in (1, N - 1):
            continue
        for _ in range(s - 1):
            x = x * x % N
            if x == N - 1:
                break
        else:
            return False
    return True


def test_wide_bench_size_sampled():
    # the benchmarked configuration: 2^30 bits from u = 2^70 + 1, B = isqrt(v) = 2^35,
    # so a bit is zero exactly when its number is prime
    l, f, n = 20, 2**49, 1024
    u, v = f * 2**(l + 1) + 1, (f + n) * 2**(l + 1)
    B = math.isqrt(v)
    assert B == 2**35
    say("wide sampled l=%d f=%d n=%d B=%d" % (l, f, n, B))
    S, c = gpu_wide(l, f, n, B)
    rng = random.Random(70)
    NB = n << l
    idx = [rng.randrange(NB) for _ in range(3000)] + list(range(64)) + list(range(NB - 64, NB))
    for j in idx:
        bit = (int(S[j >> 5]) >> (j & 31)) & 1
        assert bit == (0 if _is_probable_prime(u + 2 * j) else 1), j
    # the counts are the zero bits of each segment
    ones = np.unpackbits(S.view(np.uint8)).reshape(n, -1).sum(axis=1)
    assert np.array_equal(c.astype(np.int64), (1 << l) - ones.astype(np.int64))


def test_wide_bound_above_2_36_sampled():
    # B = 2^37 = isqrt(v) at v = 2^74: primes of up to 37 bits (the 12-bit-digit
    # remainder); every zero bit of the first 4096 and 3000 sampled bits against
    # Miller-Rabin
    l, f, n = 16, 2**57 - 8, 8
    u, v = f * 2**(l + 1) + 1, (f + n) * 2**(l + 1)
    assert v == 2**74
    B = math.isqrt(v)
    say("wide sampled l=%d f=%d n=%d B=%d" % (l, f, n, B))
    S, c = gpu_wide(l, f, n, B)
    rng = random.Random(74)
    for j in list(range(4096)) + [rng.randrange(n << l) for _ in range(3000)]:
        bit = (int(S[j >> 5]) >> (j & 31)) & 1
        assert bit == (0 if _is_probable_prime(u + 2 * j) else 1), j


def test_wide_list_and_atomic_slices_sampled():
    # 2^31 bits from u = 2^66 + 1 with B = 2^37 (above isqrt(v), so a bit is zero
    # exactly when its number is prime): the slices of primes up to about 2^36.8 list
    # their hits for the sort by table range, the later ones (fewer expected hits per
    # workgroup) OR theirs in with atomics; sampled bits against Miller-Rabin and the
    # counts against the table's zero bits
    import torch
    l, f, n = 20, 2**45, 2048
    u, v = f * 2**(l + 1) + 1, (f + n) * 2**(l + 1)
    B = 2**37
    say("wide sampled l=%d f=%d n=%d B=%d" % (l, f, n, B))
    S, c = gpu_wide(l, f, n, B)
    rng = random.Random(66)
    NB = n << l
    for j in [rng.randrange(NB) for _ in range(3000)] + list(range(64)) + list(range(NB - 64, NB)):
        bit = (int(S[j >> 5]) >> (j & 31)) & 1
        assert bit == (0 if _is_probable_prime(u + 2 * j) else 1), j
    ones = np.unpackbits(S.view(np.uint8)).reshape(n, -1).sum(axis=1)
    assert np.array_equal(c.astype(np.int64), (1 << l) - ones.astype(np.int64))
    del S, c
    torch.cuda.empty_cache()
