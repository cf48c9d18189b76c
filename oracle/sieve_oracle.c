/*
 * sieve_oracle.c -- plain, slow, single-threaded CPU reference for the odd-only
 * sieve table of Jarai & Vatai, "Cache optimized linear sieve" (2011).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle for the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant with the GPU path,
 * and the GPU path never calls it.
 *
 * What it computes (Section 1.2.1 "Input and output" and Definition 1 "Sieve
 * table, Segments" of Section 1.3):
 *   parameters l, f, n give the interval u = f*2^(l+1) + 1 .. v = (f+n)*2^(l+1);
 *   the table S has n*2^l bits, bit j stands for the odd number N_j = u + 2j;
 *   S_j = 1 (composite) iff N_j == 1, or N_j has an odd prime divisor p with
 *   3 <= p <= B and p < N_j.  With B >= isqrt(v) this is "S_j = 0 iff N_j is
 *   prime" (Section 1.4: primes up to sqrt(v) suffice).
 *   counts[t] = number of zero bits in segment t (bits t*2^l .. (t+1)*2^l - 1).
 *
 * The method reaches exactly this table faster; the oracle is the definition
 * written out: for every odd prime p <= B it sets the bit of every odd multiple
 * m*p with m >= 3 that lies in [u, v] (Section 1.1: mark the multiples of each
 * prime; Section 1.3: in the odd-only table consecutive odd multiples of p are p
 * bits apart).  No segmenting, no wheel, no buckets: those are the method's
 * speed-ups, not its result.  Bit j lives in 32-bit word j/32 at bit position
 * j%32 (least significant bit first).
 *
 * The number 1 (only present when f == 0) is set to 1 ("not prime"); the paper
 * does not say, and 1 is not a prime.
 *
 * Parity status: pinned (tests/test_oracle_pins.py: trial division on small
 * ranges, Miller-Rabin on sampled bits, known values of pi(x), Lemma 1 by
 * brute force; oracle_count_total by pi(2^22) - 1 and the sum of the counts;
 * oracle_sieve_with by oracle_sieve on prime lists running past B).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { OR_OK = 0, OR_E_ARG = -1, OR_E_RANGE = -2, OR_E_BOUND = -3, OR_E_NOMEM = -4 };

/* Odd primes 3 <= p <= B by the plain sieve of Eratosthenes (Section 1.1) over
 * the odd numbers 1..B; entry k of the byte array stands for 2k+1.  Returns the
 * number of primes written to *out (malloc'ed, caller frees) or -1. */
long oracle_odd_primes(uint64_t B, uint32_t **out)
{
    *out = NULL;
    if (B < 3) { *out = (uint32_t *)malloc(4); return *out ? 0 : -1; }
    uint64_t K = (B - 1) / 2 + 1;            /* odd numbers 1,3,...,<=B */
    unsigned char *comp = (unsigned char *)calloc(K, 1);
    if (!comp) return -1;
    for (uint64_t k = 1; k < K; ++k) {
        if (comp[k]) continue;
        uint64_t p = 2 * k + 1;
        if (p * p > B) break;
        for (uint64_t m = (p * p - 1) / 2; m < K; m += p) comp[m] = 1;
    }
    long cnt = 0;
    for (uint64_t k = 1; k < K; ++k) cnt += !comp[k];
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cnt > 0 ? cnt : 1));
    if (!pr) { free(comp); return -1; }
    long w = 0;
    for (uint64_t k = 1; k < K; ++k) if (!comp[k]) pr[w++] = (uint32_t)(2 * k + 1);
    free(comp);
    *out = pr;
    return cnt;
}

/* Validate (l, f, n, B) and return u, v, F = f*2^l, NB = n*2^l. */
static int oracle_interval(uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                           uint64_t *F, uint64_t *NB, uint64_t *u, uint64_t *v)
{
    if (l < 5 || l > 30 || n == 0) return OR_E_ARG;
    if (B < 3 || B >= ((uint64_t)1 << 32)) return OR_E_BOUND;
    u128 FF = (u128)f << l, NN = (u128)n << l;
    u128 vv = 2 * (FF + NN);
    if (vv >= ((u128)1 << 64)) return OR_E_RANGE;
    *F = (uint64_t)FF; *NB = (uint64_t)NN; *u = 2 * *F + 1; *v = (uint64_t)vv;
    return OR_OK;
}

/* Definition 1 written out, with the odd primes given: P[0..np) ascending
 * (Section 1.4's base, at least every odd prime <= B); primes above B are not
 * used.  S must hold n*2^l/32 words, counts n words. */
int oracle_sieve_with(uint32_t l, uint64_t f, uint64_t n, uint64_t B, const uint32_t *P, long np,
                      uint32_t *S, uint32_t *counts)
{
    uint64_t F, NB, u, v;
    int rc = oracle_interval(l, f, n, B, &F, &NB, &u, &v);
    if (rc) return rc;
    if (np < 0 || (np > 0 && !P)) return OR_E_ARG;
    memset(S, 0, (size_t)(NB / 32) * 4);
    for (long i = 0; i < np; ++i) {
        uint64_t p = P[i];
        if (p > B) break;
        /* smallest odd cofactor m >= 3 with m*p >= u */
        u128 m = ((u128)u + p - 1) / p;
        if (m < 3) m = 3;
        if ((m & 1) == 0) m += 1;
        u128 N = m * p;
        if (N > v) continue;
        uint64_t j = (uint64_t)((N - u) / 2);
        for (; j < NB; j += p) S[j >> 5] |= 1u << (j & 31);
    }
    if (u == 1) S[0] |= 1u;                  /* the number 1 is not prime */
    uint64_t wps = ((uint64_t)1 << l) / 32;  /* words per segment */
    for (uint64_t t = 0; t < n; ++t) {
        uint64_t ones = 0;
        for (uint64_t w = t * wps; w < (t + 1) * wps; ++w)
            ones += (uint64_t)__builtin_popcount(S[w]);
        counts[t] = (uint32_t)(((uint64_t)1 << l) - ones);
    }
    return OR_OK;
}

/* Definition 1 written out: the odd primes <= B, then oracle_sieve_with. */
int oracle_sieve(uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                 uint32_t *S, uint32_t *counts)
{
    uint64_t F, NB, u, v;
    int rc = oracle_interval(l, f, n, B, &F, &NB, &u, &v);
    if (rc) return rc;
    uint32_t *P = NULL;
    long np = oracle_odd_primes(B, &P);
    if (np < 0) return OR_E_NOMEM;
    rc = oracle_sieve_with(l, f, n, B, P, np, S, counts);
    free(P);
    return rc;
}

/* Lemma 1 (Section 2.1), in the paper's own steps: with r = f*2^(l+1) mod p the
 * unique 0 <= q < p with p | 2(f*2^l + q) + 1 is (p-r-1)/2 for even r and
 * (2p-r-1)/2 for odd r.  Here f may be any 64-bit value and l <= 63. */
uint32_t oracle_lemma1_offset(uint32_t p, uint64_t f, uint32_t l)
{
    u128 x = (u128)f << (l + 1);
    uint64_t r = (uint64_t)(x % p);
    if ((r & 1) == 0) return (uint32_t)((p - r - 1) / 2);
    return (uint32_t)((2 * (uint64_t)p - r - 1) / 2);
}

/* Lemma 2 (Section 2.2): for k*2^l <= p < (k+1)*2^l, a hit at offset q of
 * segment t is followed by a hit in segment t + k or t + k + 1.  Returns the
 * segment skip floor((q + p) / 2^l) for a hit at offset q. */
uint64_t oracle_lemma2_skip(uint32_t p, uint32_t q, uint32_t l)
{
    return ((uint64_t)q + p) >> l;
}

/* The sum of the per-segment zero-bit counts of oracle_sieve's table (the
 * table itself is discarded): the CPU baseline's unit of work.  Returns -1 on
 * error. */
long long oracle_count_total(uint32_t l, uint64_t f, uint64_t n, uint64_t B)
{
    uint64_t NBw = ((uint64_t)n << l) / 32;
    uint32_t *S = (uint32_t *)malloc((size_t)NBw * 4);
    uint32_t *c = (uint32_t *)malloc((size_t)n * 4);
    if (!S || !c) { free(S); free(c); return -1; }
    int rc = oracle_sieve(l, f, n, B, S, c);
    long long tot = 0;
    if (rc == 0) for (uint64_t t = 0; t < n; ++t) tot += c[t];
    free(S); free(c);
    return rc == 0 ? tot : -1;
}

/* Goldbach verification over a sieve table (Section 5: the program was written to
 * verify the Goldbach conjecture, and the prime table is the bulk of that work).
 * The table S is that of (l, f, n): bit j stands for the odd number u + 2j, zero
 * when it has no odd prime factor up to the table's bound (a prime, when the bound
 * reaches isqrt(v)).  The even numbers N_k = u + 1 + 2k, k = 0 .. n*2^l - 1, are
 * checked against the odd primes q <= Q in ascending order: N_k - q = u + 2(k - d)
 * with d = (q - 1)/2, which lies in the table when d <= k.
 *   minq[k]  = the least such q with d <= k and bit k - d of S zero; 0 if none;
 * and per segment t (k in [t*2^l, (t+1)*2^l)):
 *   maxq[t]  = the largest nonzero minq[k] of the segment (0 if every one is 0),
 *   argk[t]  = the least k of the segment with minq[k] == maxq[t] (k of the
 *              segment's first even number when maxq[t] == 0),
 *   fails[t] = the number of k of the segment with minq[k] == 0.
 * minq may be NULL.  Parity status: pinned (tests/test_oracle_pins.py: trial
 * division and Miller-Rabin on the numbers N - q themselves). */
int oracle_goldbach(uint32_t l, uint64_t f, uint64_t n, const uint32_t *S, uint64_t Q,
                    uint32_t *minq, uint32_t *maxq, uint64_t *argk, uint32_t *fails)
{
    uint64_t F, NB, u, v;
    int rc = oracle_interval(l, f, n, 3, &F, &NB, &u, &v);
    if (rc) return rc;
    if (Q < 3 || Q >= ((uint64_t)1 << 32)) return OR_E_BOUND;
    uint32_t *P = NULL;
    long np = oracle_odd_primes(Q, &P);
    if (np < 0) return OR_E_NOMEM;
    uint64_t seg = (uint64_t)1 << l;
    for (uint64_t t = 0; t < n; ++t) { maxq[t] = 0; argk[t] = t * seg; fails[t] = 0; }
    for (uint64_t k = 0; k < NB; ++k) {
        uint32_t best = 0;
        for (long i = 0; i < np; ++i) {
            uint64_t d = (P[i] - 1) / 2;
            if (d > k) break;                          /* N_k - q below u: not in the table */
            uint64_t j = k - d;
            if (((S[j >> 5] >> (j & 31)) & 1u) == 0) { best = P[i]; break; }
        }
        if (minq) minq[k] = best;
        uint64_t t = k >> l;
        if (best == 0) fails[t] += 1;
        else if (best > maxq[t]) { maxq[t] = best; argk[t] = k; }
    }
    free(P);
    return OR_OK;
}

/* Log-add sieve over the same interval (Section 5: circles and buckets serve a
 * wider range of sieving algorithms; a quadratic or number field sieve adds the
 * logarithm of every factor-base prime at the positions it divides instead of
 * setting a bit).  Here the factor base is the odd primes p <= B and the values
 * are the odd numbers of the interval: position j (the number N = u + 2j) collects
 *   A[j] = sum of floor(log2 p) over the odd primes p <= B that divide N
 * (every odd multiple m*p with m >= 1, so a prime p <= B in the interval counts
 * itself; each prime once whatever its power).  A[j] <= log2 N < 64, one byte.
 *   C bit j = 1 iff A[j] >= T (a smoothness candidate), same bit layout as S;
 *   counts[t] = the ones of C in segment t.
 * A may be NULL.  Parity status: pinned (tests/test_oracle_pins.py: the sums by
 * trial division, and the smooth numbers of small ranges by full factorisation). */
int oracle_logsieve(uint32_t l, uint64_t f, uint64_t n, uint64_t B, uint32_t T,
                    uint32_t *C, uint32_t *counts, uint8_t *A)
{
    uint64_t F, NB, u, v;
    int rc = oracle_interval(l, f, n, B, &F, &NB, &u, &v);
    if (rc) return rc;
    uint8_t *acc = (uint8_t *)calloc((size_t)NB, 1);
    if (!acc) return OR_E_NOMEM;
    uint32_t *P = NULL;
    long np = oracle_odd_primes(B, &P);
    if (np < 0) { free(acc); return OR_E_NOMEM; }
    for (long i = 0; i < np; ++i) {
        uint64_t p = P[i];
        uint32_t w = 0;
        while ((p >> (w + 1)) != 0) ++w;            /* floor(log2 p) */
        u128 m = ((u128)u + p - 1) / p;              /* smallest m with m*p >= u */
        if ((m & 1) == 0) m += 1;                    /* odd multiples only */
        u128 N = m * p;
        if (N > v) continue;
        for (uint64_t j = (uint64_t)((N - u) / 2); j < NB; j += p) acc[j] = (uint8_t)(acc[j] + w);
    }
    free(P);
    memset(C, 0, (size_t)(NB / 32) * 4);
    for (uint64_t j = 0; j < NB; ++j)
        if (acc[j] >= T) C[j >> 5] |= 1u << (j & 31);
    uint64_t wps = ((uint64_t)1 << l) / 32;
    for (uint64_t t = 0; t < n; ++t) {
        uint64_t ones = 0;
        for (uint64_t w = t * wps; w < (t + 1) * wps; ++w) ones += (uint64_t)__builtin_popcount(C[w]);
        counts[t] = (uint32_t)ones;
    }
    if (A) memcpy(A, acc, (size_t)NB);
    free(acc);
    return OR_OK;
}

/* Odd primes 3 <= p <= B for B up to 2^40 (64-bit values), by the same plain sieve
 * of Eratosthenes as oracle_odd_primes.  Returns the count or -1. */
long long oracle_odd_primes64(uint64_t B, uint64_t **out)
{
    *out = NULL;
    if (B < 3 || B > ((uint64_t)1 << 40)) { *out = (uint64_t *)malloc(8); return (B < 3 && *out) ? 0 : -1; }
    uint64_t K = (B - 1) / 2 + 1;
    unsigned char *comp = (unsigned char *)calloc(K, 1);
    if (!comp) return -1;
    for (uint64_t k = 1; k < K; ++k) {
        if (comp[k]) continue;
        uint64_t p = 2 * k + 1;
        if (p * p > B) break;
        for (uint64_t m = (p * p - 1) / 2; m < K; m += p) comp[m] = 1;
    }
    long long cnt = 0;
    for (uint64_t k = 1; k < K; ++k) cnt += !comp[k];
    uint64_t *pr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cnt > 0 ? cnt : 1));
    if (!pr) { free(comp); return -1; }
    long long w = 0;
    for (uint64_t k = 1; k < K; ++k) if (!comp[k]) pr[w++] = 2 * k + 1;
    free(comp);
    *out = pr;
    return cnt;
}

/* Definition 1 for intervals beyond 2^64 (Section 5: sieving with primes above 32
 * bits): f is given as two 64-bit halves (f = f_hi * 2^64 + f_lo), so
 * u = f*2^(l+1) + 1 and v = (f+n)*2^(l+1) may reach 2^128 - 2^(l+1); the bound
 * B may reach 2^40.  The table is the same: bit j is set iff u + 2j == 1 or it has
 * an odd prime divisor p <= B with p < u + 2j (every odd multiple m*p, m >= 3). */
int oracle_sieve_wide(uint32_t l, uint64_t f_lo, uint64_t f_hi, uint64_t n, uint64_t B,
                      uint32_t *S, uint32_t *counts)
{
    if (l < 5 || l > 30 || n == 0) return OR_E_ARG;
    if (B < 3 || B > ((uint64_t)1 << 40)) return OR_E_BOUND;
    u128 f = ((u128)f_hi << 64) | f_lo;
    if (f >> (127 - l)) return OR_E_RANGE;
    u128 F = f << l, NB128 = (u128)n << l;
    if (NB128 >> 40) return OR_E_ARG;
    u128 vv = 2 * (F + NB128);
    if (vv < 2 * F) return OR_E_RANGE;                  /* wrapped past 2^128 */
    uint64_t NB = (uint64_t)NB128;
    u128 u = 2 * F + 1, v = vv;
    memset(S, 0, (size_t)(NB / 32) * 4);
    uint64_t *P = NULL;
    long long np = oracle_odd_primes64(B, &P);
    if (np < 0) return OR_E_NOMEM;
    for (long long i = 0; i < np; ++i) {
        u128 p = P[i];
        /* the first odd multiple m*p >= u, m >= 3, as a distance from u (u + p
         * itself may pass 2^128 when v is near it) */
        u128 d = (p - u % p) % p;             /* u + d: the first multiple of p >= u */
        if ((d & 1) != 0) d += p;             /* u odd: the first odd one */
        if (u <= p && u + d == p) d += 2 * p; /* m = 1: p itself stays */
        if (d / 2 >= NB) continue;
        uint64_t j = (uint64_t)(d / 2);
        for (; j < NB; j += (uint64_t)p) S[j >> 5] |= 1u << (j & 31);
    }
    free(P);
    if (u == 1) S[0] |= 1u;
    uint64_t wps = ((uint64_t)1 << l) / 32;
    for (uint64_t t = 0; t < n; ++t) {
        uint64_t ones = 0;
        for (uint64_t w = t * wps; w < (t + 1) * wps; ++w) ones += (uint64_t)__builtin_popcount(S[w]);
        counts[t] = (uint32_t)(((uint64_t)1 << l) - ones);
    }
    return OR_OK;
}
