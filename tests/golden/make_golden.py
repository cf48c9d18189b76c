"""Writes the full-size expected values used by the GPU parity tests.

Calls only the CPU oracle (oracle/oracle.py).  For each workload it stores the
per-segment zero-bit counts and the SHA-256 of the table bytes (little-endian
uint32 words), so the GPU tests can check every bit of a 512 MiB table without
holding a second copy.

Workloads (interval parameters of Section 1.2.1):
  interval_1e12    : l=20, n=4096, f=floor((10^12 - 2^32)/2^21), B = isqrt(v)
  interval_1e12_b6 : the same interval with the literal bound B = 10^6 (partial sieve)
  interval_2p60    : l=20, n=4096, f=2^39-2048 (centred at 2^60), B = 2^30
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
    }


def main(names):
    W = workloads()
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
