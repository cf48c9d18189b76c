"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

Every table bit and every per-segment count must be identical (integer work, one
correct answer).  Small cases compare whole tables with the oracle; the
full-size workloads compare per-segment counts and the SHA-256 of the whole
table with values the oracle wrote (tests/golden/make_golden.py).
"""
import collections
import json
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_util import say, gpu_sieve, sha256_words, first_diff

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def check_case(l, f, n, B, tune=None, **kw):
    say("case l=%d f=%d n=%d B=%d tune=%s" % (l, f, n, B, tune))
    S, c = gpu_sieve(l, f, n, B, tune=tune, **kw)
    So, co = O.sieve(l, f, n, B)
    assert first_diff(S, So) is None, ("table", l, f, n, B, tune, first_diff(S, So))
    assert np.array_equal(c, co), ("counts", l, f, n, B, tune)
    return S, c


def test_small_config_pi_2_22():
    # l=15, f=0, n=64 sieves 1..2^22 with primes <= 2048: pi(2^22) = 295947
    S, c = check_case(15, 0, 64, 2048)
    assert int(c.sum()) + 1 == 295947
    assert int(c[0]) == 6541


@pytest.mark.parametrize("case", [
    (5, 0, 1, 3), (5, 0, 1, 13), (6, 0, 3, 17), (10, 0, 4, 1000), (11, 0, 16, 3),
    (12, 5, 7, 61), (16, 0, 1, 65535), (20, 0, 2, 65536), (20, 0, 1, 65537),
    (18, 1, 3, 2000), (13, 1000, 9, 200003),
    # 2^20-bit tiles from 1 with small bounds: the primes themselves stay unmarked
    (20, 0, 1, 61), (20, 0, 1, 60), (20, 0, 3, 1000),
])
def test_edge_cases(case):
    check_case(*case)


def test_near_2_64_partial_sieve():
    # v = (f+n)*2^21 = 2^64 - 2^22: the largest interval end the interface allows
    check_case(20, 2**43 - 2, 1, 10**6)
    check_case(20, 2**43 - 3, 2, 3)


def test_near_2_64_bucket_path():
    # large primes (p >= 2^20 at the default tuning) with first hits computed from
    # a 64-bit start near 2^63 (G0 = f*2^20)
    check_case(20, 2**43 - 4, 3, 3 * 10**6)
    # the bucket path forced on with a small medium bound: 16- and 32-bit entries,
    # several chunks per launch
    check_case(20, 2**43 - 3, 2, 10**6, tune={"tile_log2": 15, "medium_log2": 11, "bins_log2": 8})
    check_case(17, 2**46 - 40, 32, 2 * 10**6,
               tune={"tile_log2": 17, "medium_log2": 14, "bins_log2": 8, "bin_log2": 17, "groups": 96})


@pytest.mark.parametrize("case", [
    (20, 2**43 - 4, 3, 10**7),               # near 2^64
    (18, 12345, 10, 5 * 10**6),              # every sparse prime starts past v (p^2 rule)
    (16, 0, 64, 10**7),                      # from the number 1
    (20, (10**15) >> 21, 4, 2 * 10**7),
    (20, (10**12) >> 21, 40, 2**31 + 11),    # the largest bound class
    (13, (10**15) >> 14, 385, 2 * 10**7),    # 97 bins of the hit sort, the last one partial
])
def test_sparse_large_primes_direct(case):
    # large primes at least as long as the table take the sparse path (one hit at
    # most, sorted by bin and OR-ed in after the tile kernel, counts taken again);
    # also with tiles shorter than the segments (per-tile count atomics, then the
    # recount), and turned off (the bucket path)
    l, f, n, B = case
    check_case(l, f, n, B, tune={"sparse": 2})
    check_case(l, f, n, B, tune={"sparse": 2, "tile_log2": 15})
    check_case(l, f, n, B, tune={"sparse": 1})


def test_sparse_path_random_cases():
    # seeded random tables whose large primes reach at least the table length, so
    # that the sparse path runs (tables of 2^21.5..2^25 bits at starts up to 2^62,
    # bounds from the table length to 2^28, ragged bin counts, default and small
    # tiles), every one against the oracle
    rng = random.Random(1111)
    for k in range(16):
        l = rng.choice([13, 15, 17, 18, 20])
        nb = int(2 ** rng.uniform(21.5, 25))
        n = max(1, nb >> l)
        nb = n << l
        f = rng.randrange(0, 2 ** (61 - l))
        B = rng.randrange(nb, 2**28)
        u, v = O.interval(l, f, n)
        tune = {"sparse": 2} if k % 2 == 0 else {"sparse": 2, "tile_log2": 15}
        check_case(l, f, n, B, tune=tune)


def test_sparse_path_wide_window_golden():
    # a 2^30-bit table from 2^62 with every prime below 2^32: the sparse primes
    # (2^30 <= p < 2^32; 1.49e8 of them with 3.52e7 hits, none from those above
    # 2^31, whose squares lie past the table) take 1024 bins of 2^20 bits; the
    # sparse path and the bucket path both against the oracle's golden (counts of
    # every segment and the SHA-256 of the table)
    import torch
    from paper_1111_3297_amd import api
    g = _golden("interval_2p62_w30")
    l, f, n, B = g["l"], g["f"], g["n"], g["B"]
    pr = api.Primes(B)
    for tune in ({"sparse": 2}, {"sparse": 1}):
        say("sparse wide window", l, f, n, B, tune)
        S, c = gpu_sieve(l, f, n, B, tune=tune, primes=pr)
        assert [int(x) for x in c] == g["counts"], tune
        assert sha256_words(S) == g["S_sha256"], tune
    del pr
    torch.cuda.empty_cache()


def test_planned_scratch_equals_held_scratch():
    # the planning pass (sieve_sieve_scratch_bytes) gives exactly the device bytes a
    # fresh context holds after the call: the sparse path, the bucket path, medium
    # primes only
    from paper_1111_3297_amd import api
    for (l, f, n, B, tune) in [(20, 2**43 - 65, 64, 2**32 - 1, None), (20, 2**43 - 65, 64, 2**32 - 1, {"sparse": 1}),
                               (20, (10**12) >> 21, 40, 2**31 + 11, None), (20, (10**14) >> 21, 8, 10**6, None)]:
        pr = api.Primes(B)
        ctx = api.Context()
        planned = ctx.sieve_scratch_bytes(l, f, n, B, tune=tune, primes=pr)
        S, c = api.alloc(l, n)
        ctx.sieve(l, f, n, B, S, c, tune=tune, primes=pr)
        ctx.check_device_errors()
        assert ctx.scratch_bytes() == planned, (l, f, n, B, tune)


@pytest.mark.parametrize("groups", [1024, 4096])
def test_bucket_fill_workgroup_counts(groups):
    # the bucket-fill workgroup counts the batch autotuner may pick, on the plain path
    l, f, n = 20, (10**14) >> 21, 24
    check_case(l, f, n, math.isqrt(O.interval(l, f, n)[1]), tune={"groups": groups})


def test_random_small_with_tunings():
    rng = random.Random(20111111)
    tunings = [None,
               {"tile_log2": 13, "medium_log2": 9, "wave_log2": 9, "bins_log2": 8, "groups": 64},
               {"tile_log2": 14, "medium_log2": 12, "wave_log2": 9, "wheel_log2": 10, "bins_log2": 9},
               {"tile_log2": 17, "medium_log2": 14, "wave_log2": 10, "wheel_log2": 12},
               {"tile_log2": 15, "medium_log2": 16, "wave_log2": 9, "wheel_log2": 9, "bins_log2": 10, "groups": 128},
               {"tile_log2": 17, "medium_log2": 15, "wave_log2": 9, "bins_log2": 9, "bin_log2": 17},
               {"tile_log2": 14, "medium_log2": 11, "wave_log2": 9, "bins_log2": 8, "bin_log2": 14},
               {"tile_log2": 16, "medium_log2": 13, "bins_log2": 10, "bin_log2": 16, "groups": 200, "ranges": 1},
               {"tile_log2": 15, "medium_log2": 12, "bins_log2": 9, "groups": 100, "ranges": 4}]
    for k in range(40):
        l = rng.choice([5, 7, 11, 13, 15, 16, 17])
        n = rng.randint(1, max(1, (1 << 21) >> l))
        e = rng.choice([0, 3, 6, 9, 12, 15, 18])
        f = (10**e) >> (l + 1) if e else 0
        f += rng.randint(0, 50)
        u, v = O.interval(l, f, n)
        r = math.isqrt(v)
        B = rng.choice([r, r, max(3, r // 7), min(r, 5 * 10**5) if r > 3 else 3])
        B = max(3, min(B, 2**24))
        tune = tunings[k % len(tunings)]
        if tune is not None and tune["tile_log2"] > l + 10:   # per-tile count slots must fit LDS
            tl = l + 10
            tune = dict(tune, tile_log2=tl, medium_log2=min(max(tune["medium_log2"], tl - 4), tl + 1))
            tune["wave_log2"] = 9
            tune["wheel_log2"] = max(9, min(tune.get("wheel_log2", tl - 4), tune["medium_log2"]))
            if "bin_log2" in tune:
                tune["bin_log2"] = tl
        check_case(l, f, n, B, tune=tune)


def test_invalid_tuning_rejected():
    from paper_1111_3297_amd import api, _lib
    S, c = api.alloc(5, 4)
    with pytest.raises(_lib.SieveError):
        api.Context().sieve(5, 0, 4, 100, S, c, tune={"tile_log2": 17})


def test_multi_chunk_and_bucket_path():
    # small bins force several bucket-fill chunks per launch and many large primes
    t = {"tile_log2": 13, "medium_log2": 9, "wave_log2": 9, "bins_log2": 8, "groups": 96}
    check_case(13, (10**12) >> 14, 1 << 10, 10**6, tune=t)   # 2^23 bits, 4 chunks
    check_case(15, (10**15) >> 16, 1 << 8, 2 * 10**6, tune={"tile_log2": 15, "medium_log2": 11, "bins_log2": 8})
    # 32-bit bucket entries: one bin per tile
    check_case(17, (10**14) >> 18, 1 << 6, 3 * 10**6,
               tune={"tile_log2": 17, "medium_log2": 14, "bins_log2": 8, "bin_log2": 17, "groups": 80})
    # eight bin ranges of one bin each
    check_case(15, (10**13) >> 16, 8, 10**6, tune={"tile_log2": 15, "medium_log2": 11, "bins_log2": 8, "groups": 64,
                                                     "ranges": 8})


@pytest.mark.parametrize("case", [
    # 2^20-bit tiles over short segments: one word per lane at write-out (l = 12, no
    # 17..47 masks) and four words per lane with the masks (l = 13)
    (12, (10**9) >> 13, 512, 40000), (13, (10**9) >> 14, 256, 40000),
    # the 17..47 masks need every prime up to 47
    (20, 0, 2, 46), (20, 0, 2, 47), (20, 1, 2, 53), (20, (10**10) >> 21, 3, 47),
])
def test_write_out_paths_on_2p20_tiles(case):
    l, f, n, B = case
    check_case(l, f, n, B, tune={"tile_log2": 20})


def test_carried_rows_across_tiles():
    # more tiles than workgroups, so each workgroup carries the next-hit offsets of
    # the largest medium primes from tile to tile; primes above sqrt(u) start at p^2
    # inside the interval (beyond a workgroup's first tile for some of them)
    check_case(20, (4 * 10**10) >> 21, 600, 300007)
    # from 1: p^2 starts of every carried class fall inside later tiles of the runs
    check_case(20, 0, 600, 300007)
    # tiles of eight segments with a ragged last tile
    check_case(17, (10**11) >> 18, 4801, 250000, tune={"tile_log2": 20})


def test_prime_table_matches_oracle():
    import torch
    from paper_1111_3297_amd import api
    for B in [3, 5, 13, 17, 1000, 65535, 65536, 65537, 10**6, 2**24 + 17, 10**8 + 7]:
        say("prime table B=%d" % B)
        pr = api.Primes(B)
        got = pr.to_tensor().cpu().numpy().view(np.uint32)
        torch.cuda.synchronize()
        want = O.odd_primes(B)
        assert pr.count == len(want), B
        assert np.array_equal(got, want), B
        pr.close()


def test_shared_table_and_contexts_on_two_streams():
    import torch
    from paper_1111_3297_amd import api
    pr = api.Primes(10**7)
    jobs = [(16, (10**13) >> 17, 64, 10**7 - 1), (17, (10**13) >> 18, 32, 3 * 10**6)]
    outs = []
    ctxs = [api.Context(), api.Context()]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for (l, f, n, B), ctx, st in zip(jobs, ctxs, streams):
        say("two-stream job", l, f, n, B)
        S, c = api.alloc(l, n)
        with torch.cuda.stream(st):
            ctx.sieve(l, f, n, B, S, c, primes=pr, stream=st)
        outs.append((S, c))
    torch.cuda.synchronize()
    for (l, f, n, B), (S, c) in zip(jobs, outs):
        So, co = O.sieve(l, f, n, B)
        assert first_diff(S.cpu().numpy().view(np.uint32), So) is None
        assert np.array_equal(c.cpu().numpy().view(np.uint32), co)
    for ctx in ctxs:
        ctx.check_device_errors()


def test_bucket_contents_match_corollary_1():
    # Corollary 1 / Theorem 1 (Section 2.3): every hit of every large prime in the
    # chunk appears exactly once, in the bucket of its bin, with its in-bin offset.
    from paper_1111_3297_amd import api
    l, f, n, B = 13, (10**10) >> 14, 256, 200003
    for tune in ({"tile_log2": 13, "medium_log2": 10, "wave_log2": 9, "bins_log2": 8, "groups": 64, "bin_log2": 13},
                 {"tile_log2": 17, "medium_log2": 14, "wave_log2": 9, "bins_log2": 8, "groups": 64, "bin_log2": 16},
                 {"tile_log2": 15, "medium_log2": 11, "wave_log2": 9, "bins_log2": 8, "groups": 64, "bin_log2": 15}):
        _check_buckets(l, f, n, B, tune)


def _check_buckets(l, f, n, B, tune):
    from paper_1111_3297_amd import api
    say("bucket dump", l, f, n, B, tune)
    d = api.debug_buckets(l, f, n, B, tune=tune)
    b, cb = d["bin_log2"], d["chunk_bits"]
    F = f << l
    primes = [int(p) for p in O.odd_primes(B) if p >= (1 << tune["medium_log2"])]
    assert d["nlarge"] == len(primes)
    want = [[] for _ in range(len(d["bin_start"]) - 1)]
    for p in primes:
        q = ((p - 1) // 2 - F) % p
        j = q
        gsq = (p * p - 1) // 2
        if gsq > F + j:
            j = gsq - F
        while j < cb:
            want[j >> b].append(j & ((1 << b) - 1))
            j += p
    # each hit at least once; padding only repeats hits of the same bin, within the bound
    bs = d["bin_start"]
    for k in range(len(want)):
        got = collections.Counter(int(x) for x in d["entries"][bs[k]:bs[k + 1]])
        need = collections.Counter(want[k])
        assert set(got) == set(need) and all(got[v] >= c for v, c in need.items()), k
        assert sum(got.values()) <= len(want[k]) + d["pad_per_bin"], k


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % name)
    with open(path) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name", ["interval_1e12", "interval_1e12_b6", "interval_2p60", "interval_3win",
                                  "serve_req71", "serve_req6388", "interval_2p64_top"])
def test_full_size_against_oracle_golden(name):
    g = _golden(name)
    say("full size", name, g["l"], g["f"], g["n"], g["B"])
    S, c = gpu_sieve(g["l"], g["f"], g["n"], g["B"])
    assert [int(x) for x in c] == g["counts"]
    assert sha256_words(S) == g["S_sha256"]


@pytest.mark.parametrize("B", [2133783848, 4294967295])
def test_prime_table_against_oracle_golden(B):
    # the largest bound the serving stream uses, and the largest the interface allows
    import hashlib
    import torch
    from paper_1111_3297_amd import api
    g = _golden("primes_%d" % B)
    say("prime table golden B=%d" % B)
    pr = api.Primes(B)
    assert pr.count == g["count"], (pr.count, g["count"])
    got = pr.to_tensor().cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    assert int(got[-1]) == g["max"]
    assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == g["sha256"]
    pr.close()
