"""Autotuner for the batched launch and the plain sieve.

The tuning knobs of include/sieve.h (tile size, medium/wheel class bounds, bucket
layout) cannot change any result -- the table is unique given (l, f, n, B) -- so
the tuner simply times candidate settings on the workload itself with HIP events
on the launch stream and keeps the fastest.  Results are cached in a JSON file
keyed by a coarse workload signature, so a serving process tunes once per
workload class.
"""
import json
import math
import os
import time

import torch

from . import api

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_ENV = "SIEVE_AUTOTUNE_CACHE"
BUILTIN = os.path.join(HERE, "autotune_builtin.json")


def default_cache_path():
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "sieve_mi355x_autotune.json"))


# Version of the candidate sets below: part of every cache key, so that entries
# timed over an older set of candidates are tuned again.
TUNER_VERSION = 2


def signature(l, reqs):
    """Coarse workload class: tuner version, segment size, request count, total
    table bits and largest bound, each rounded to a power of two."""
    bits = sum(n << l for (_, n, _) in reqs)
    bmax = max(B for (_, _, B) in reqs)
    return "v%d|l=%d|nreq=%d|bits=2^%d|B=2^%d" % (TUNER_VERSION, l, 1 << max(0, (len(reqs) - 1).bit_length()),
                                                  max(0, bits - 1).bit_length(), max(0, bmax - 1).bit_length())


def candidates(l, bmax):
    """Tile sizes 2^17..2^20 (the LDS-resident segment), each with the medium bound
    at the tile size or twice it and two wheel-class bounds."""
    out = []
    for L in (20, 19, 18, 17):
        if L > l + 10:
            continue
        for M in (L, L + 1):
            for Wb in (L - 7, L - 6):
                if Wb < 9 or Wb > M:
                    continue
                out.append({"tile_log2": L, "medium_log2": M, "wheel_log2": Wb})
    return out


def bucket_candidates():
    """Bucket-layout variants tried around the best tile setting: the number of
    bucket-fill workgroups (a batch shares them out over its requests by estimated
    work; the library's default is 2048)."""
    return [{"groups": 1024}, {"groups": 4096}]


def _load(path):
    data = {}
    for p in (BUILTIN, path):
        if p and os.path.exists(p):
            try:
                with open(p) as fh:
                    data.update(json.load(fh))
            except (OSError, ValueError):
                pass
    return data


def _store(path, key, rec):
    data = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                data = json.load(fh)
        except (OSError, ValueError):
            data = {}
    data[key] = rec
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(ctx, primes, l, outs, tune, repeats=2):
    """Mean milliseconds of one sieve_batch over `repeats` runs (after one warm-up)."""
    stream = torch.cuda.current_stream()
    ctx.batch(primes, l, outs, tune=tune)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(repeats):
        ctx.batch(primes, l, outs, tune=tune)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / repeats


def tune_batch(primes, l, outs, ctx=None, cache_path=None, force=False, repeats=2, log=None):
    """Best tune (dict) for sieve_batch on these requests.  outs: list of
    (f, n, B, S, counts) exactly as Context.batch takes them."""
    cache_path = cache_path or default_cache_path()
    key = signature(l, [(f, n, B) for (f, n, B, _, _) in outs])
    cached = _load(cache_path)
    if not force and key in cached:
        return dict(cached[key]["tune"])
    ctx = ctx or api.Context()
    bmax = max(B for (_, _, B, _, _) in outs)
    results = []
    for t in candidates(l, bmax):
        ms = time_batch(ctx, primes, l, outs, t, repeats)
        results.append((ms, t))
        if log:
            log("autotune %s %.3f ms" % (t, ms))
    results.sort(key=lambda x: x[0])
    best_ms, best = results[0]
    if bmax >= (1 << best["medium_log2"]):
        # large primes: the bucket-fill workgroup mapping around the best tile setting
        for extra in bucket_candidates():
            t = dict(best, **extra)
            ms = time_batch(ctx, primes, l, outs, t, repeats)
            results.append((ms, t))
            if log:
                log("autotune %s %.3f ms" % (t, ms))
        results.sort(key=lambda x: x[0])
        best_ms, best = results[0]
    _store(cache_path, key, {"tune": best, "ms": best_ms, "when": time.strftime("%Y-%m-%d %H:%M:%S"),
                             "tried": [{"tune": t, "ms": m} for (m, t) in results]})
    return dict(best)


def tune_plain(l, f, n, B, primes=None, ctx=None, cache_path=None, force=False, repeats=2, log=None):
    """Best tune for one interval (same candidates, timed with sieve_ctx_sieve)."""
    cache_path = cache_path or default_cache_path()
    key = "plain|" + signature(l, [(f, n, B)])
    cached = _load(cache_path)
    if not force and key in cached:
        return dict(cached[key]["tune"])
    ctx = ctx or api.Context()
    primes = primes or api.Primes(B)
    S, c = api.alloc(l, n)
    stream = torch.cuda.current_stream()
    results = []
    for t in candidates(l, B):
        ctx.sieve(l, f, n, B, S, c, tune=t, primes=primes)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(repeats):
            ctx.sieve(l, f, n, B, S, c, tune=t, primes=primes)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / repeats
        results.append((ms, t))
        if log:
            log("autotune plain %s %.3f ms" % (t, ms))
    results.sort(key=lambda x: x[0])
    _store(cache_path, key, {"tune": results[0][1], "ms": results[0][0],
                             "tried": [{"tune": t, "ms": m} for (m, t) in results]})
    return dict(results[0][1])
