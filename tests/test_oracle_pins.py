"""Pins for the CPU oracle: values fixed by mathematics, not by the oracle itself.

* brute-force trial division of every represented number on tiny intervals
  (Definition 1, Section 1.3, including the partial sieve B < isqrt(v));
* published values of pi(x) (tests/golden/pi_values.txt);
* deterministic Miller-Rabin on every bit of mid-size intervals and on random
  samples of large ones;
* Lemma 1 (Section 2.1) against the brute-force least offset;
* Lemma 2 (Section 2.2): the skip after a hit of a prime with k*2^l <= p < (k+1)*2^l
  is k or k+1 segments.
"""
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime_mr(n):
    """Deterministic Miller-Rabin for n < 3.3e24 with the first twelve primes as bases."""
    if n < 2:
        return False
    for p in MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def smallest_odd_factor(N):
    d = 3
    while d * d <= N:
        if N % d == 0:
            return d
        d += 2
    return N


def brute_bits(l, f, n, B):
    """Definition 1 by trial division: S_j = 1 iff N_j == 1 or N_j has an odd prime
    divisor p <= B with p < N_j (the least odd factor is that divisor if any is)."""
    u, _ = O.interval(l, f, n)
    out = np.zeros(n << l, dtype=np.uint8)
    for j in range(n << l):
        N = u + 2 * j
        if N == 1:
            out[j] = 1
            continue
        q = smallest_odd_factor(N)
        out[j] = 1 if (q <= B and q < N) else 0
    return out


def bits_of(S):
    return np.unpackbits(S.view(np.uint8), bitorder="little")


def test_brute_force_small_intervals():
    rng = random.Random(7)
    cases = [(5, 0, 1, 3), (5, 0, 2, 13), (5, 0, 8, 17), (6, 0, 4, 61), (5, 1, 1, 3),
             (7, 3, 5, 1000), (10, 0, 4, 64), (8, 64, 3, 11), (9, 17, 2, 3)]
    for _ in range(40):
        l = rng.randint(5, 10)
        f = rng.randint(0, 64)
        n = rng.randint(1, 8)
        u, v = O.interval(l, f, n)
        r = math.isqrt(v)
        B = rng.choice([r, max(3, r // 3), 3, 5, 13, 17, 31, r + 50])
        cases.append((l, f, n, B))
    for (l, f, n, B) in cases:
        S, c = O.sieve(l, f, n, B)
        got = bits_of(S)
        want = brute_bits(l, f, n, B)
        assert np.array_equal(got, want), (l, f, n, B)
        seg = (1 << l)
        for t in range(n):
            assert c[t] == seg - int(want[t * seg:(t + 1) * seg].sum())


def pi_table():
    vals = []
    with open(os.path.join(HERE, "golden", "pi_values.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                vals.append((int(line[0]), int(line[1]), len(line) > 2 and line[2] == "golden"))
    return vals


def test_pi_values_from_published_table():
    vals = [(x, pi) for (x, pi, big) in pi_table() if not big]
    for x, pi in vals:
        # base-prime generator: odd primes <= x plus the prime 2
        assert len(O.odd_primes(x)) + 1 == pi, x
    # the table itself: f = 0 and B = isqrt(v) gives zero bits exactly at the odd
    # primes, so sum(counts) + 1 (for the prime 2) = pi(v)
    for (l, n, x) in [(15, 64, 4194304), (16, 8, 1048576), (10, 32, 65536)]:
        _, c = O.sieve(l, 0, n, math.isqrt(x))
        pi = dict(vals)[x]
        assert int(c.sum()) + 1 == pi


def test_miller_rabin_every_bit_mid_interval():
    # 2^16 numbers just above 10^12 and just below 2^62: every bit checked
    for (l, f, n) in [(12, 10**12 // 2**13, 8), (12, 2**61 // 2**13 - 8, 8)]:
        u, v = O.interval(l, f, n)
        S, c = O.sieve(l, f, n, math.isqrt(v))
        bits = bits_of(S)
        for j in range(n << l):
            assert bits[j] == (0 if is_prime_mr(u + 2 * j) else 1), (l, f, j)


def test_miller_rabin_sampled_large_interval():
    # a 2^25-number interval near 10^15 with the full base (B = isqrt(v))
    l, n = 20, 16
    f = 10**15 // 2**21
    u, v = O.interval(l, f, n)
    S, c = O.sieve(l, f, n, math.isqrt(v))
    bits = bits_of(S)
    rng = np.random.default_rng(11)
    for j in rng.integers(0, n << l, 3000):
        j = int(j)
        assert bits[j] == (0 if is_prime_mr(u + 2 * j) else 1)
    # every zero bit in the first 2^12 bits is a prime (density check on a block)
    zeros = np.flatnonzero(bits[:4096] == 0)
    assert all(is_prime_mr(u + 2 * int(j)) for j in zeros)
    # prime number theorem sanity: density ~ 2/ln(N) over odd numbers
    expect = (n << l) * 2 / math.log(u)
    assert abs(int(c.sum()) - expect) < 0.01 * expect


def test_partial_sieve_marks_only_small_factors():
    # B < isqrt(v): a one bit must have an odd factor <= B; a zero bit must not
    l, f, n, B = 12, 10**9 // 2**13, 4, 1000
    u, v = O.interval(l, f, n)
    S, _ = O.sieve(l, f, n, B)
    bits = bits_of(S)
    primes = [p for p in O.odd_primes(B)]
    rng = np.random.default_rng(3)
    for j in rng.integers(0, n << l, 2000):
        N = u + 2 * int(j)
        has = any(N % p == 0 and p < N for p in primes)
        assert bits[int(j)] == (1 if has else 0)


def test_lemma1_offset_brute_force():
    rng = random.Random(5)
    primes = [int(p) for p in O.odd_primes(5000)]
    for _ in range(3000):
        p = rng.choice(primes)
        l = rng.randint(0, 40)
        f = rng.randint(0, (1 << 63) >> l) if rng.random() < 0.7 else rng.randint(0, 100)
        q = O.lemma1_offset(p, f, l)
        assert 0 <= q < p
        assert (2 * ((f << l) + q) + 1) % p == 0
        # uniqueness: no smaller offset divides
        if p < 200:
            assert all((2 * ((f << l) + r) + 1) % p != 0 for r in range(q))


def test_lemma2_skip_is_k_or_k_plus_1():
    rng = random.Random(9)
    primes = [int(p) for p in O.odd_primes(1 << 22)]
    for _ in range(5000):
        l = rng.randint(5, 20)
        p = rng.choice(primes)
        k = p >> l
        q = rng.randrange(1 << l)
        assert O.lemma2_skip(p, q, l) in (k, k + 1)


def test_invalid_arguments_raise():
    with pytest.raises(O.OracleError):
        O.sieve(4, 0, 1, 3)          # l < 5
    with pytest.raises(O.OracleError):
        O.sieve(10, 0, 0, 3)         # n == 0
    with pytest.raises(O.OracleError):
        O.sieve(10, 0, 1, 2)         # B < 3
    with pytest.raises(O.OracleError):
        O.sieve(10, 0, 1, 1 << 32)   # B >= 2^32
    with pytest.raises(O.OracleError):
        O.sieve(20, (1 << 43), 1, 3)  # v >= 2^64


def test_count_total_equals_sum_of_counts():
    # the CPU baseline's unit of work: the total of the table's per-segment counts;
    # 1..2^22 with primes <= 2048 leaves the odd primes below 2^22, pi(2^22) - 1
    assert O.count_total(15, 0, 64, 2048) == 295946
    rng = random.Random(5)
    for _ in range(6):
        l = rng.choice([5, 9, 12, 14])
        f = rng.randint(0, 10**6)
        n = rng.randint(1, 9)
        u, v = O.interval(l, f, n)
        B = max(3, math.isqrt(v) // rng.choice([1, 3]))
        assert O.count_total(l, f, n, B) == int(O.sieve(l, f, n, B)[1].astype(np.int64).sum())


def test_sieve_with_given_primes_uses_only_those_up_to_B():
    # a prime list running past B sieves exactly as the primes <= B alone
    P = O.odd_primes(5000)
    for (l, f, n, B) in [(10, 0, 4, 13), (10, 0, 4, 3000), (12, 12345, 3, 997), (14, 10**6, 2, 4999)]:
        S0, c0 = O.sieve(l, f, n, B)
        S1, c1 = O.sieve_with(l, f, n, B, P)
        assert np.array_equal(S0, S1) and np.array_equal(c0, c1), (l, f, n, B)


def test_prime_table_goldens_match_published_pi():
    # the oracle's odd primes <= 2^32 - 1 (written once by make_golden.py) number
    # pi(2^32) - 1; below 2^31 + 1 they number pi(2^31) - 1
    import json
    pub = {x: pi for (x, pi, _) in pi_table()}
    g = json.load(open(os.path.join(HERE, "golden", "primes_4294967295.json")))
    assert g["count"] + 1 == pub[4294967296] and g["max"] == 4294967291
    # 2133783848 lies below 2^31: its count is at most pi(2^31) - 1 and the table is
    # the prefix of the 2^32 one (checked on the GPU); 104459685 = pi(2133783848) - 1
    # was counted independently of this oracle
    g2 = json.load(open(os.path.join(HERE, "golden", "primes_2133783848.json")))
    assert g2["count"] == 104459685 and g2["count"] + 1 <= pub[2147483648]


def test_goldbach_records_match_published_table():
    # the table of 1 .. 2^22 (primes <= 2048): the running maxima of the least q
    # over the even numbers are the published Goldbach records
    S, _ = O.sieve(15, 0, 64, 2048)
    minq, maxq, argk, fails = O.goldbach(15, 0, 64, S, 2048)
    want = []
    with open(os.path.join(HERE, "golden", "goldbach_records.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if line:
                want.append((int(line[0]), int(line[1])))
    rec, best = [], 0
    for k in np.flatnonzero(minq):
        if minq[k] > best:
            best = int(minq[k])
            rec.append((2 + 2 * int(k), best))
    assert rec == want
    # only N = 2 and N = 4 (= 2 + 2, the odd primes cannot reach it) fail
    assert int(fails.sum()) == 2 and list(np.flatnonzero(minq == 0)) == [0, 1]


def _least_q_brute(N, k, Q, prime):
    q = 3
    while q <= Q and (q - 1) // 2 <= k:
        if prime(q) and prime(N - q):
            return q
        q += 2
    return 0


def test_goldbach_against_trial_division():
    rng = random.Random(11)
    for _ in range(8):
        l = rng.choice([5, 7, 9, 10])
        n = rng.randint(1, 6)
        f = rng.choice([0, rng.randint(0, 3000)])
        u, v = O.interval(l, f, n)
        S, _ = O.sieve(l, f, n, max(3, math.isqrt(v)))
        Q = rng.choice([3, 17, 200, 1000])
        minq, maxq, argk, fails = O.goldbach(l, f, n, S, Q)
        prime = lambda x: x >= 2 and smallest_odd_factor(x) == x if x % 2 else x == 2
        for k in range(n << l):
            assert minq[k] == _least_q_brute(u + 1 + 2 * k, k, Q, prime), (l, f, n, Q, k)
        # the per-segment summary follows from the per-number values
        seg = 1 << l
        for t in range(n):
            m = minq[t * seg:(t + 1) * seg]
            assert fails[t] == int((m == 0).sum())
            assert maxq[t] == int(m.max())
            if maxq[t]:
                assert argk[t] == t * seg + int(np.flatnonzero(m == maxq[t])[0])


def test_goldbach_partial_table_and_large_numbers():
    # a partial table (B < isqrt(v)): the check reads "no odd prime factor <= B"
    l, f, n, B = 8, 7000, 3, 31
    u, v = O.interval(l, f, n)
    S, _ = O.sieve(l, f, n, B)
    minq, _, _, _ = O.goldbach(l, f, n, S, 500)
    rough = lambda x: all(x % p for p in range(3, B + 1, 2) if smallest_odd_factor(p) == p and p < x)
    for k in range(n << l):
        N = u + 1 + 2 * k
        q = 3
        want = 0
        while q <= 500 and (q - 1) // 2 <= k:
            if smallest_odd_factor(q) == q and rough(N - q):
                want = q
                break
            q += 2
        assert minq[k] == want, k
    # near 10^12 with the full bound: sampled even numbers by Miller-Rabin
    l, f, n = 12, (10**12) >> 13, 4
    u, v = O.interval(l, f, n)
    S, _ = O.sieve(l, f, n, math.isqrt(v))
    minq, _, _, fails = O.goldbach(l, f, n, S, 5000)
    rng = random.Random(3)
    for k in rng.sample(range(3000, n << l), 300):
        assert minq[k] == _least_q_brute(u + 1 + 2 * k, k, 5000, is_prime_mr), k
    assert int(fails[1:].sum()) == 0


def _odd_prime_factors(N):
    out, d = [], 3
    while N % 2 == 0:
        N //= 2
    while d * d <= N:
        if N % d == 0:
            out.append(d)
            while N % d == 0:
                N //= d
        d += 2
    if N > 1:
        out.append(N)
    return out


def test_logsieve_sums_by_trial_division():
    rng = random.Random(17)
    for _ in range(10):
        l = rng.choice([5, 6, 8, 10])
        n = rng.randint(1, 5)
        f = rng.choice([0, rng.randint(0, 5000), rng.randint(10**6, 10**7)])
        u, v = O.interval(l, f, n)
        B = rng.choice([3, 13, 97, 1000, max(3, math.isqrt(v))])
        T = rng.randint(0, 40)
        C, c, A = O.logsieve(l, f, n, B, T)
        for j in range(n << l):
            N = u + 2 * j
            want = sum(p.bit_length() - 1 for p in _odd_prime_factors(N) if p <= B)
            assert A[j] == want, (l, f, n, B, N)
            assert ((int(C[j >> 5]) >> (j & 31)) & 1) == (want >= T)
        assert [int(x) for x in c] == [int(sum(bin(int(w)).count("1") for w in C[t << (l - 5):(t + 1) << (l - 5)]))
                                       for t in range(n)]


def test_logsieve_smooth_numbers():
    # with T = 0 every bit is one; with B >= N a prime counts its own floor(log2);
    # an odd squarefree N whose prime factors are all <= B has A(N) >= log2 N minus
    # its number of prime factors (each floor loses less than one)
    l, f, n = 10, 0, 4
    u, v = O.interval(l, f, n)
    C, c, A = O.logsieve(l, f, n, v, 0)
    assert int(c.sum()) == n << l
    for j in range(1, n << l):
        N = u + 2 * j
        fs = _odd_prime_factors(N)
        if len(fs) == 1 and fs[0] == N:
            assert A[j] == N.bit_length() - 1
        prod = 1
        for p in fs:
            prod *= p
        if prod == N:
            assert A[j] >= math.log2(N) - len(fs)
    assert A[0] == 0    # the number 1


def test_sieve_wide_agrees_below_2_64_and_miller_rabin_above():
    # below 2^64 the wide oracle is the plain one
    for (l, f, n, B) in [(10, 0, 3, 100), (12, (10**15) >> 13, 2, 10**5), (20, 2**43 - 3, 1, 3000)]:
        S0, c0 = O.sieve(l, f, n, B)
        S1, c1 = O.sieve_wide(l, f, n, B)
        assert np.array_equal(S0, S1) and np.array_equal(c0, c1)
    # just past 2^64 with the bound isqrt(v), a little above 2^32: zero bits are exactly
    # the primes (deterministic Miller-Rabin below 3.3e24)
    l, n = 12, 1
    f = (2**64 + 2**45) >> (l + 1)
    u, v = O.interval(l, f, n)
    B = math.isqrt(v)
    assert B > 2**32 + 4000
    S, c = O.sieve_wide(l, f, n, B)
    bits = np.unpackbits(S.view(np.uint8), bitorder="little")
    for j in range(n << l):
        assert bool(bits[j]) == (not is_prime_mr(u + 2 * j)), j


def test_sieve_wide_near_2_128_by_trial_division():
    # v = 2^128 - 2^11: every sampled bit is 1 exactly when an odd prime p <= B divides
    # its number (p below it); the residues come from the number's two 64-bit halves
    # and 2^64 mod p, independently of the oracle's arithmetic
    l, n, B = 10, 8, 2**20 + 7
    f = 2**117 - 1 - n
    u, v = f * 2**(l + 1) + 1, (f + n) * 2**(l + 1)
    assert v == 2**128 - 2**11 and B > v - u
    S, c = O.sieve_wide(l, f, n, B)
    bits = np.unpackbits(S.view(np.uint8), bitorder="little")
    P = O.odd_primes(B).astype(np.uint64)
    t64 = (np.uint64(2**64 - 1) % P + np.uint64(1)) % P
    rng = np.random.default_rng(128)
    idx = sorted(set(rng.integers(0, n << l, 300).tolist()) | set(range(40)) | set(range((n << l) - 40, n << l)))
    for j in idx:
        N = u + 2 * j
        hi, lo = np.uint64(N >> 64), np.uint64(N & (2**64 - 1))
        r = ((hi % P) * t64 + lo % P) % P
        assert bool(bits[j]) == bool((r == 0).any()), j
    assert int(c.sum()) == (n << l) - int(bits.sum())


def test_odd_primes64_below_2_32_is_odd_primes():
    for B in (3, 1000, 10**6 + 3):
        assert np.array_equal(O.odd_primes64(B), O.odd_primes(B).astype(np.uint64))
