"""CPU checks of the benchmark's work accounting: the algorithmic and the executed
mark counts behind the roofline figures, against brute force on small intervals."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _primes(n):
    s = np.ones(n + 1, bool)
    s[:2] = False
    for i in range(2, int(n ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0]


def _brute(P, u, v, tile_log2):
    alg = exe = 0
    for p in P:
        if p < 17:
            continue
        for N in range(max(u, p * p), v + 1):
            if N % p or N % 2 == 0:
                continue
            alg += 1
            m = N // p
            if p >= 53 and (p >= (1 << (tile_log2 - 3)) or (m % 3 and m % 5)):
                exe += 1
    return alg, exe


def test_mark_counts_match_brute_force():
    P = _primes(3000)
    P = P[P >= 3]
    for (u, v, L) in [(1, 120000, 15), (1000001, 1130000, 16), (12345679, 12405679, 17), (3, 9000, 13)]:
        alg, exe = _brute(P, u, v, L)
        assert bench.marks_algorithmic(P, u, v) == alg, (u, v)
        assert bench.marks_executed(P, u, v, tile_log2=L) == exe, (u, v, L)


def test_kernel_hash_ignores_comments(tmp_path):
    src = os.path.join(ROOT, "paper_1111_3297_amd", "csrc")
    d = tmp_path / "paper_1111_3297_amd" / "csrc"
    d.mkdir(parents=True)
    for name in ("kernels.inc", "logsieve.inc", "sieve.hip"):
        text = open(os.path.join(src, name)).read()
        (d / name).write_text("// an added comment\n" + text.replace("\n", "\n  ", 3) + "\n/* trailing */\n")
    h0 = bench.kernel_source_hash()
    old = bench.ROOT
    try:
        bench.ROOT = str(tmp_path)
        h1 = bench.kernel_source_hash()
        (d / "kernels.inc").write_text((d / "kernels.inc").read_text() + "\nint changed;\n")
        h2 = bench.kernel_source_hash()
    finally:
        bench.ROOT = old
    assert h0 == h1 and h1 != h2


def test_log_adds_match_brute_force():
    P = _primes(2000)
    P = P[P >= 3]
    for (u, v) in [(1, 20000), (99999, 130000), (10**9 + 1, 10**9 + 40000)]:
        want = sum(1 for p in P for N in range(u, v + 1) if N % 2 and N % p == 0)
        assert bench.log_adds(P, u, v) == want, (u, v)


def test_sparse_counts_match_brute_force():
    # sparse large primes (p at least the table length) and those of them with a
    # hit: an odd multiple of p in [max(u, p^2), v]
    P = _primes(40000)
    P = P[P >= 3].astype(np.uint32)
    for (l, f, n) in [(10, 12345, 4), (12, 0, 2), (11, 999, 3)]:
        nb = n << l
        u = (f << (l + 1)) + 1
        v = u + 2 * (nb - 1)
        sp = [int(p) for p in P if p >= nb]
        hits = 0
        for p in sp:
            lo = max(u, p * p)
            m = -(-lo // p)
            if m % 2 == 0:
                m += 1
            hits += m * p <= v
        assert bench.sparse_counts(P, l, f, n) == (len(sp), hits), (l, f, n)
    # the largest 32-bit primes (p^2 near 2^64) against tables near 2^62 and 2^64
    big = np.array([4294967291, 4294967279, 4294967231, 4294967197, 4294967189, 4294967161, 3037000493,
                    3037000453, 2147483647, 2147483629], dtype=np.uint32)
    for (l, f, n) in [(20, 2**43 - 65, 64), (20, 2**41, 64), (16, 2**46 - 7, 3)]:
        nb = n << l
        u = (f << (l + 1)) + 1
        v = u + 2 * (nb - 1)
        hits = 0
        for p in (int(x) for x in big):
            lo = max(u, p * p)
            m = -(-lo // p)
            if m % 2 == 0:
                m += 1
            hits += m * p <= v
        assert bench.sparse_counts(big, l, f, n) == (len(big), hits), (l, f, n)
