"""Writes the full-size expected values used by the GPU parity tests.

Calls only the CPU oracle (oracle/oracle.py).  For each workload it stores the
per-segment zero-bit counts and the SHA-256 of the table bytes (little-endian
uint32 words), so the GPU tests can check every bit of a 512 MiB table without
holding a second copy.

Workloads (interval parameters of Section 1.2.1):
  interval_1e12    : l=20, n=4096, f=floor((10^12 - 2^32)/2^21), B = isqrt(v)
  interval_1e12_b6 : the same interval with the literal bound B = 10^6 (partial sieve)
  interval_2p60    : l=20, n=4096, f=2^39-2048 (centred at 2^60), B = 2^30
  interval_3win    : l=20, n=5120 from 512 segments below interval_1e12's start,
                     B = isqrt(v): three launch windows of 2^31, 2^31 and 2^30 bits
  serve_req71      : request 71 of the seeded serving stream (the first with
                     B > 2^30): l=20, n=128, B = isqrt(v) = 1907618081
  serve_req6388    : request 6388 of the stream, its largest bound:
                     B = isqrt(v) = 2133783848
  interval_2p64_top: l=20, n=64 ending at v = 2^64 - 2^21, B = isqrt(v) = 2^32 - 1
  interval_2p62_w30: l=20, f=2^41 (u = 2^62 + 1), n=1024 (2^30 bits), B = 2^32 - 1,
                     every 32-bit prime: those from 2^30 on hit the table at most once
                     each, those above 2^31 not at all (their squares lie past v)
  wide_2p66        : beyond 2^64 (128-bit f): l=16, f=2^49-128, n=128 ending at
                     v = 2^66, B = 2^33 = isqrt(v) (primes above 32 bits sieve)
  wide_b32         : l=14, f=2^90+12345, n=64, B = 2^32 - 1 (every 32-bit prime)
  wide_top         : l=12, f=2^115-41, n=40 ending at v = 2^128 - 2^13,
                     B = 2^32 + 2^28 + 1 (partial; primes on both sides of 2^32)
  wide_u2p64       : l=20, f=2^43 (u = 2^64 + 1), n=16, B = 2^32 + 2^30 + 3
  wide_2p66_2g     : l=20, f=2^45-2048, n=2048 (2^31 bits) ending at v = 2^66,
                     B = 2^33: about one hit per two primes above 2^32
  wide_2p68        : l=16, f=2^51-128, n=128 ending at v = 2^68, B = 2^34 = isqrt(v)
  primes_2133783848, primes_4294967295: the odd primes <= B (count and SHA-256
                     of the ascending little-endian uint32 array)
  batch_1234       : the 256 interval requests of the seeded batch workload
                     (paper_1111_3297_amd/workloads.py), B = isqrt(v) each
  serve_99         : every request of the seeded serving stream (60 s at 200/s),
                     B = isqrt(v) each: zero-bit total and the first 16 hex digits
                     of the SHA-256 of its counts and of its table
Run: python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402

F_1E12 = (10**12 - 2**32) // 2**21


def workloads():
    u, v = O.interval(20, F_1E12, 4096)
    return {
        "interval_1e12": (20, F_1E12, 4096, math.isqrt(v)),
        "interval_1e12_b6": (20, F_1E12, 4096, 10**6),
        "interval_2p60": (20, 2**39 - 2048, 4096, 2**30),
        "interval_3win": (20, F_1E12 - 512, 5120, math.isqrt(O.interval(20, F_1E12 - 512, 5120)[1])),
        "serve_req71": (20, 1735213635173, 128, 1907618081),
        "serve_req6388": (20, 2171055560302, 128, 2133783848),
        "interval_2p64_top": (20, 2**43 - 65, 64, 2**32 - 1),
        "interval_2p62_w30": (20, 2**41, 1024, 2**32 - 1),
    }


def wide_workloads():
    return {
        "wide_2p66": (16, 2**49 - 128, 128, 2**33),
        "wide_b32": (14, 2**90 + 12345, 64, 2**32 - 1),
        "wide_top": (12, 2**115 - 41, 40, 2**32 + 2**28 + 1),
        "wide_u2p64": (20, 2**43, 16, 2**32 + 2**30 + 3),
        "wide_2p66_2g": (20, 2**45 - 2048, 2048, 2**33),
        "wide_2p68": (16, 2**51 - 128, 128, 2**34),
    }


def wide_golden(name):
    l, f, n, B = wide_workloads()[name]
    t = time.time()
    S, c = O.sieve_wide(l, f, n, B)
    dt = time.time() - t
    rec = {"name": name, "l": l, "f": str(f), "n": n, "B": B,
           "u": str(f * 2**(l + 1) + 1), "v": str((f + n) * 2**(l + 1)),
           "S_sha256": hashlib.sha256(S.tobytes()).hexdigest(),
           "total_zero_bits": int(c.sum()), "counts": [int(x) for x in c],
           "oracle_seconds": round(dt, 1)}
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh)
    print(name, rec["total_zero_bits"], round(dt, 1), "s", flush=True)


def prime_golden(B):
    """The odd primes <= B: their count and the SHA-256 of the uint32 array."""
    t = time.time()
    P = O.odd_primes(B)
    rec = {"name": "primes_%d" % B, "B": B, "count": int(len(P)), "max": int(P[-1]),
           "sha256": hashlib.sha256(P.astype("<u4").tobytes()).hexdigest(), "oracle_seconds": round(time.time() - t, 1)}
    with open(os.path.join(HERE, rec["name"] + ".json"), "w") as fh:
        json.dump(rec, fh)
    print(rec["name"], rec["count"], rec["oracle_seconds"], "s", flush=True)


_P = None


def _serve_one(job):
    global _P
    if _P is None:
        _P = O.odd_primes(job[4])
    rid, f, n, B, _ = job
    S, c = O.sieve_with(20, f, n, B, _P)
    return rid, int(c.astype("int64").sum()), hashlib.sha256(c.astype("<u4").tobytes()).hexdigest()[:16], \
        hashlib.sha256(S.tobytes()).hexdigest()[:16]


def serve_golden(name="serve_99", procs=6):
    """Every request of the seeded serving stream, in worker processes that each
    hold the oracle's prime list up to the stream's largest bound."""
    import multiprocessing as mp
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from paper_1111_3297_amd import workloads as WL
    stream = WL.serving_stream(99, 200.0, 60.0)
    jobs = []
    for rid, (t, f21, n21, kind) in enumerate(stream):
        jobs.append((rid, f21, n21, math.isqrt(O.interval(20, f21, n21)[1])))
    bmax = max(j[3] for j in jobs)
    order = sorted(jobs, key=lambda j: -(j[2] + j[3] / 2**21))   # longest first
    t = time.time()
    out = [None] * len(jobs)
    with mp.Pool(procs) as pool:
        for k, (rid, tot, ch, sh) in enumerate(pool.imap_unordered(_serve_one, [j + (bmax,) for j in order], 4)):
            out[rid] = [tot, ch, sh]
            if k % 500 == 0:
                print("serve golden", k, "of", len(jobs), round(time.time() - t, 1), "s", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump({"name": name, "l": 20, "seed": 99, "rate": 200.0, "seconds": 60.0, "count": len(jobs),
                   "fields": ["total", "counts_sha256_16", "S_sha256_16"], "requests": out,
                   "oracle_seconds": round(time.time() - t, 1)}, fh, separators=(",", ":"))
    print(name, sum(r[0] for r in out), round(time.time() - t, 1), "s", flush=True)


def batch_golden(name="batch_1234"):
    """The 256-request batch (seed 1234): per request the oracle's zero-bit total and
    the SHA-256 of its counts and of its table, with B = isqrt(v) per request."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from paper_1111_3297_amd import workloads as WL
    out = []
    t = time.time()
    for f21, n21 in WL.batch_requests(1234, 256):
        u, v = O.interval(20, f21, n21)
        B = math.isqrt(v)
        S, c = O.sieve(20, f21, n21, B)
        out.append({"f": f21, "n": n21, "B": B, "total": int(c.sum()),
                    "counts_sha256": hashlib.sha256(c.astype("<u4").tobytes()).hexdigest(),
                    "S_sha256": hashlib.sha256(S.tobytes()).hexdigest()})
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump({"name": name, "l": 20, "requests": out, "oracle_seconds": round(time.time() - t, 1)}, fh)
    print(name, sum(r["total"] for r in out), round(time.time() - t, 1), "s", flush=True)


def main(names):
    W = workloads()
    if names == ["batch_1234"]:
        batch_golden()
        return
    if names == ["serve_99"]:
        serve_golden()
        return
    for name in [x for x in names if x.startswith("primes_")]:
        prime_golden(int(name.split("_")[1]))
    for name in [x for x in names if x.startswith("wide_")]:
        wide_golden(name)
    names = [x for x in names if not x.startswith(("primes_", "wide_"))] if names else None
    if names == []:
        return
    for name in names or list(W):
        l, f, n, B = W[name]
        t = time.time()
        S, c = O.sieve(l, f, n, B)
        dt = time.time() - t
        rec = {"name": name, "l": l, "f": f, "n": n, "B": B,
               "u": O.interval(l, f, n)[0], "v": O.interval(l, f, n)[1],
               "S_sha256": hashlib.sha256(S.tobytes()).hexdigest(),
               "total_zero_bits": int(c.sum()), "counts": [int(x) for x in c],
               "oracle_seconds": round(dt, 1)}
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(rec, fh)
        print(name, rec["total_zero_bits"], round(dt, 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
