/*
 * sieve.h -- C ABI of the MI355X (gfx950) segmented odd-only sieve of Eratosthenes.
 *
 * The library computes the sieve table of Definition 1 (Section 1.3) of Jarai &
 * Vatai, "Cache optimized linear sieve" (2011), for the interval of Section 1.2.1:
 *
 *     u = f * 2^(l+1) + 1,   v = (f + n) * 2^(l+1),
 *
 * a table S of n * 2^l bits in which bit j stands for the odd number u + 2j;
 * bit j is 1 ("sieved out") iff u + 2j == 1 or u + 2j has an odd prime divisor
 * p <= B with p < u + 2j, and 0 otherwise.  With B >= isqrt(v) the zero bits are
 * exactly the odd primes in [u, v] (Section 1.4: the base is the primes up to
 * sqrt(v)).  B < isqrt(v) is allowed and gives the partial sieve just defined.
 * Bit j is bit (j % 32) of 32-bit word j / 32 (least significant bit first).
 *
 * counts[t] is the number of zero bits in segment t, i.e. in bits
 * t*2^l .. (t+1)*2^l - 1 (Definition 1's segments S^(t)).
 *
 * Conventions for every entry point:
 *  - Return value: SIEVE_OK (0) on success, a negative sieve_status otherwise.
 *    Nothing is enqueued when an argument check fails.  Faults that happen on the
 *    device later surface as SIEVE_E_HIP from a later call or from
 *    sieve_check_device_errors().
 *  - Pointers named *_dev are device pointers (HIP device memory, e.g. the data
 *    pointer of a torch.cuda tensor); the caller owns them and keeps them alive
 *    until the stream work has finished.  Host pointers are only read during the
 *    call.
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.  Work
 *    is enqueued on it and the call returns without synchronising, except where
 *    an entry point says otherwise.
 *  - Validity: 5 <= l <= 20 (whole 32-bit words per segment), n >= 1,
 *    v = (f+n)*2^(l+1) < 2^64, 3 <= B < 2^32 (the paper's 32-bit sieving primes,
 *    Section 5).
 *  - The library never calls back into Python and never throws.
 */
#ifndef SIEVE_MI355X_H
#define SIEVE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIEVE_OK = 0,
    SIEVE_E_ARG = -1,     /* l, n, a pointer or a tuning field is out of range        */
    SIEVE_E_RANGE = -2,   /* v = (f+n)*2^(l+1) does not fit in 64 bits                */
    SIEVE_E_BOUND = -3,   /* B < 3, B >= 2^32, or B above the prime table's bound     */
    SIEVE_E_NOMEM = -4,   /* device allocation failed                                */
    SIEVE_E_HIP = -5,     /* a HIP runtime call failed (see sieve_last_hip_error)     */
    SIEVE_E_BUDGET = -6,  /* batch scratch would exceed the caller's byte budget      */
    SIEVE_E_DEVICE = -7,  /* a kernel reported a violated invariant (bucket overflow) */
    SIEVE_E_SCRATCH = -8  /* the request needs more than the static scratch array holds */
} sieve_status;

/* Tuning knobs.  A zero field means "library default".  None of them can change
 * the table or the counts (the result is unique given l, f, n, B); they only
 * move work between kernels.
 *   tile_log2   log2 of the LDS-resident tile in bits (the paper's cache segment,
 *               Section 1.2); 13..20.  Default: l clamped to [15, 20].
 *   medium_log2 primes below 2^medium_log2 are sieved per tile in LDS (Section
 *               2.1 "medium primes"); primes at or above it take the bucket path
 *               (Sections 2.2-2.5).  tile_log2-4 .. tile_log2+1.  Default tile_log2.
 *   wave_log2   medium primes below 2^wave_log2 are sieved by a whole wavefront
 *               each, those below 2^wheel_log2 by eight lanes each (one per
 *               residue of the 3-5 wheel, Section 3.2.1), the rest by one lane
 *               each (walking the wheel when a prime has eight or more hits per
 *               tile): the GPU form of the per-hit-count grouping of Section
 *               3.2.2.  9 <= wave_log2 <= wheel_log2 <= medium_log2.
 *               Defaults 9 and min(tile_log2-7, medium_log2) (at least 9).
 *   bins_log2   log2 of the number of large-prime buckets per chunk, 8..15.
 *   groups      workgroups of the bucket-fill kernels, 64..4096; default 2048.
 *               Each takes a contiguous slice of the large primes of equal
 *               estimated work.  With ranges given, a chunk's workgroups are split
 *               over its ranges (groups rounded down to a multiple of ranges);
 *               by default every range gets groups workgroups.
 *   ranges      the bins of a chunk are filled in this many ranges (1, 2, 4 or 8;
 *               0, the default: two for chunks of 1024 bins or more, else one).
 *               Fewer bins per scatter workgroup leave fewer partly written
 *               cache lines, at the cost of visiting every large prime once per
 *               range; the per-bin counts are taken once for the whole chunk.
 *   bin_log2    log2 of one bucket's width in bits, min(tile_log2,16)..tile_log2.
 *               Up to 16 a hit is stored as a 16-bit in-bucket offset, above 16
 *               as a 32-bit one.
 *   sparse      large primes at least as long as a launch window (2^31 bits, or
 *               the whole table when shorter) hit it at most once.  0 (default)
 *               or 2: they skip the bucket fill; after the tile kernel has
 *               written the window their hits are computed, counting-sorted by
 *               table range and OR-ed in (then the counts are taken again).  1
 *               keeps them in the buckets.  sieve_ctx_sieve and sieve_init only;
 *               batches keep every large prime in the buckets.
 *   wide_list, wide_slot_log2, wide_sort_hits: sieve_wide only.  On tables of
 *               at most 2^31 bits every prime above 2^32 hits at most once; a
 *               slice of those primes either lists its hits (each workgroup in a
 *               slot of 2^wide_slot_log2 entries, 6..13, default 12; hits beyond
 *               it are OR-ed into S with atomics) for a sort by table range
 *               whose workgroups gather about wide_sort_hits expected hits
 *               (16..65536, default 7600; a workgroup takes at most 8192, any
 *               beyond go in with atomics), or ORs every hit into S with atomics.
 *               wide_list 0 (default): list where a slice's workgroups expect at
 *               least 96 hits; 1: never; 2: every slice.
 */
typedef struct {
    uint32_t tile_log2;
    uint32_t medium_log2;
    uint32_t wave_log2;
    uint32_t bins_log2;
    uint32_t groups;
    uint32_t bin_log2;
    uint32_t wheel_log2;
    uint32_t ranges;
    uint32_t sparse;
    uint32_t wide_list;
    uint32_t wide_slot_log2;
    uint32_t wide_sort_hits;
    uint32_t reserved[2];
} sieve_tune;

/* One interval of a batch: the interval of Section 1.2.1 with parameters
 * (l, f, n) where l is the batch's l; S_dev holds n*2^l/32 words and counts_dev
 * n words; B is this request's sieving bound (3 <= B <= the prime table's bound). */
typedef struct {
    uint64_t f;
    uint64_t n;
    uint64_t B;
    uint32_t *S_dev;
    uint32_t *counts_dev;
} sieve_req;

typedef struct sieve_ctx sieve_ctx;        /* library-owned device workspace        */
typedef struct sieve_primes sieve_primes;  /* library-owned device sieving-prime table */

/* --- one-shot entry point (Section 1.2.1 parameters l, f, n plus the bound B) ---
 * Sieves the n segments of 2^l bits starting at segment f with the odd primes
 * 3 <= p <= B, writing S_dev (n*2^l/32 uint32 words) and counts_dev (n uint32).
 * Generates the sieving primes on the device (Section 1.4 initialization),
 * computes the first offsets (Lemma 1), sieves each LDS tile with the pre-sieved
 * pattern of 3..13, the medium primes (Section 2.1) and the bucketed large-prime
 * hits (Sections 2.2-2.5), and writes each tile out with its popcount; large
 * primes at least as long as a 2^31-bit launch window (one hit there at most) have
 * their hits sorted by table range and OR-ed in after that (see sparse below), and
 * the counts are then taken again.
 * Uses the calling thread's default context (one per device). */
int sieve_init(uint32_t l, uint64_t f, uint64_t n, uint64_t B,
               uint32_t *S_dev, uint32_t *counts_dev, void *stream);

/* Same as sieve_init on an explicit context with explicit tuning (tune may be
 * NULL).  Calls on one context are ordered by the context; contexts are
 * independent, so two contexts may run on two streams at once. */
int sieve_ctx_create(sieve_ctx **out);
int sieve_ctx_destroy(sieve_ctx *ctx);   /* synchronises the context's last stream */
int sieve_ctx_sieve(sieve_ctx *ctx, uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                    uint32_t *S_dev, uint32_t *counts_dev, const sieve_tune *tune,
                    void *stream);

/* --- shared sieving-prime table (Section 1.4, Definition 2: the base) ---
 * Builds the odd primes 3 <= p <= B on the device and SYNCHRONISES the stream
 * once, so that the prime count is known on the host. */
int sieve_primes_create(uint64_t B, void *stream, sieve_primes **out);
int sieve_primes_destroy(sieve_primes *pr);
/* Number of primes in the table and its bound B. */
int sieve_primes_info(const sieve_primes *pr, uint64_t *count, uint64_t *bound);
/* Copies the first min(count, cap) primes (ascending uint32) to dst_dev. */
int sieve_primes_copy(const sieve_primes *pr, uint32_t *dst_dev, uint64_t cap, void *stream);

/* --- sieve with a shared table (no prime generation inside the call) --- */
int sieve_ctx_sieve_with(sieve_ctx *ctx, const sieve_primes *pr, uint32_t l, uint64_t f,
                         uint64_t n, uint64_t B, uint32_t *S_dev, uint32_t *counts_dev,
                         const sieve_tune *tune, void *stream);

/* --- batched persistent launch (Section 5: sieving combined with parallel
 * processing, here many intervals of Section 1.2.1 in one launch) ---
 * Sieves every request of reqs[0..nreq) (all with segment size 2^l) against the
 * one shared table pr: one offset kernel, one bucket fill and one persistent tile
 * kernel for the whole batch, whose workgroups take (request, run of up to 16
 * consecutive tiles) work items from a device queue in request order, the runs
 * shortening as the queue drains (single tiles at its end).  Each request's table
 * and counts are the same as sieve_init would give for it alone. */
int sieve_batch(sieve_ctx *ctx, const sieve_primes *pr, uint32_t l, const sieve_req *reqs,
                size_t nreq, const sieve_tune *tune, void *stream);
/* --- device memory accounting (for admission control by a byte budget) ---
 * sieve_batch_scratch_bytes: the device bytes a fresh context holds after
 * sieve_batch on these requests (bucket storage and per-request state; not the
 * caller's S and counts, not the prime table).  The bucket part follows the hit
 * count of Sections 2.2-2.3 (a prime p hits a span of s bits about s/p times,
 * summed over the large primes).  Computed by a planning pass of sieve_batch that
 * allocates and enqueues nothing; it queries the current device's attributes.
 * S_dev / counts_dev of reqs are not read and may be NULL.
 * sieve_sieve_scratch_bytes: the same for sieve_ctx_sieve_with (pr given) or
 * sieve_ctx_sieve (pr NULL: the context's own prime table up to B included).
 * A context's buffers only grow, so a call on a used context adds at most these
 * bytes to what sieve_ctx_scratch_bytes reports for it. */
int sieve_batch_scratch_bytes(const sieve_primes *pr, uint32_t l, const sieve_req *reqs,
                              size_t nreq, const sieve_tune *tune, uint64_t *bytes);
int sieve_sieve_scratch_bytes(const sieve_primes *pr, uint32_t l, uint64_t f, uint64_t n,
                              uint64_t B, const sieve_tune *tune, uint64_t *bytes);
/* Device bytes the context's scratch buffers hold now. */
int sieve_ctx_scratch_bytes(sieve_ctx *ctx, uint64_t *bytes);
/* Synchronises the context's last stream and frees all its scratch buffers (the
 * next call allocates again).  Clears the context's device error word. */
int sieve_ctx_trim(sieve_ctx *ctx);
/* Device bytes of a prime table. */
int sieve_primes_bytes(const sieve_primes *pr, uint64_t *bytes);

/* --- Goldbach check over a sieve table (Section 5: the verification the program
 * was written for, for which the prime table is the bulk of the work) ---
 * S_dev is the table of (l, f, n) as sieve_init writes it (n*2^l/32 words; a zero
 * bit stands for an odd number with no odd prime factor up to the table's bound,
 * i.e. a prime when the bound reached isqrt(v)).  The even numbers
 * N_k = u + 1 + 2k, k = 0 .. n*2^l - 1, are checked against the odd primes
 * q <= Q of the table pr (Q <= its bound), ascending: N_k - q is table bit k - d
 * with d = (q - 1)/2, available when d <= k.
 *   minq[k]  (optional, minq_dev may be NULL; n*2^l uint32) = the least such q
 *            whose bit is zero, 0 if none;
 * per segment t (the numbers k in [t*2^l, (t+1)*2^l)), n entries each:
 *   maxq_dev[t]  = the largest nonzero minq of the segment (0 if none),
 *   argk_dev[t]  = the least k of the segment with that minq (t*2^l if maxq is 0),
 *   fails_dev[t] = the numbers of the segment with minq 0 (N - q < u for every q
 *                  that works, or no q <= Q works: a counterexample candidate
 *                  up to Q when d_max <= k).
 * All outputs are caller-owned device memory, written on stream.  The context's
 * scratch holds one 8-byte maximum per segment.  Errors: SIEVE_E_ARG (null
 * pointers, l, n, more than 2^44 table bits), SIEVE_E_RANGE, SIEVE_E_BOUND (Q < 3 or
 * Q above the prime table's bound). */
int sieve_goldbach(sieve_ctx *ctx, const sieve_primes *pr, uint32_t l, uint64_t f, uint64_t n,
                   const uint32_t *S_dev, uint64_t Q, uint32_t *maxq_dev, uint64_t *argk_dev,
                   uint32_t *fails_dev, uint32_t *minq_dev, void *stream);

/* --- log-add sieve over the interval (Section 5: circles and buckets for a wider
 * range of sieving algorithms, where a quadratic or number field sieve adds the
 * logarithm of each factor-base prime at the positions it divides) ---
 * Positions are the odd numbers N = u + 2j of the interval (l, f, n); the factor
 * base is the odd primes p <= B (the table pr, or the context's own table up to B
 * when pr is NULL); each adds floor(log2 p) at every odd multiple m*p, m >= 1 (each
 * prime once, whatever its power).  A sum is at most log2 N < 64.
 *   C_dev      (n*2^l/32 uint32 words, bit layout of S): bit j = 1 iff the sum at
 *              u + 2j is at least T (0 <= T <= 255), a smoothness candidate;
 *   counts_dev (n uint32): the ones of C per segment;
 *   A_dev      (optional, NULL or n*2^l bytes): the sums themselves.
 * Tiles of 2^tile_log2 positions (14..17, default 17; tune may be NULL) hold their
 * byte sums in LDS; primes below the tile size are walked per tile, larger ones go
 * through the buckets of Sections 2.2-2.5 with their weight in the entry (groups
 * and ranges of the tune apply to that fill, by default 4 ranges sharing 1024
 * workgroups; the other fields are ignored).
 * Errors as sieve_ctx_sieve, SIEVE_E_ARG also for T > 255 or a tile size out of
 * range; bucket overflow sets the device error word. */
int sieve_logsieve(sieve_ctx *ctx, const sieve_primes *pr, uint32_t l, uint64_t f, uint64_t n,
                   uint64_t B, uint32_t T, uint32_t *C_dev, uint32_t *counts_dev, uint8_t *A_dev,
                   const sieve_tune *tune, void *stream);

/* --- intervals beyond 2^64 (Section 5: sieving with primes of more than 32 bits,
 * the extension the paper names for its 32-bit implementation) ---
 * Definition 1 for the interval (l, f, n) with a 128-bit f = f_hi*2^64 + f_lo:
 * u = f*2^(l+1) + 1 and v = (f+n)*2^(l+1) with 2^64 < u and v < 2^128 (the segment
 * boundary 2^64 splits an interval that crosses it into a sieve_init part and a
 * sieve_wide part).  The odd primes 3 <= p <= B sieve, with 3 <= B <= 2^40 (B may
 * reach 2^32 and beyond: B >= isqrt(v) makes S an exact prime table up to
 * v = 2^80).  Outputs as sieve_init: S_dev (n*2^l/32 words, bit j <-> u + 2j),
 * counts_dev (n words).  Every p < 2^41 is below sqrt(u), so the p^2 start rule
 * never applies.  The primes up to min(B, 2^32 - 1) take the path of
 * sieve_ctx_sieve (the context's own table, first offsets from the 128-bit start);
 * the primes above 2^32 are produced in slices of 2^30 odd numbers by sieving
 * those numbers on the device (the context keeps one slice, 132 MiB at most);
 * their hits (fewer than one per prime on average) are sorted by table range and
 * OR-ed into S a range at a time, or OR-ed into S directly (see the wide_* fields
 * of sieve_tune; tune may be NULL); the counts are then taken again from S.  The
 * sort keeps one slice's hit slots (16 KiB per workgroup by default, 256 MiB) and
 * the call's sorted hits with their bin headers (about 5 B per hit: 0.7 GB at
 * v = 2^71 with B = 2^35) in the context as well.
 * Validity: 5 <= l <= 20, 1 <= n < 2^31, n*2^l < 2^40.  Errors: SIEVE_E_ARG (null
 * pointers, l, n, a wide_* field out of range), SIEVE_E_RANGE (u below 2^64 or v
 * not below 2^128), SIEVE_E_BOUND (B < 3 or B > 2^40). */
int sieve_wide(sieve_ctx *ctx, uint32_t l, uint64_t f_lo, uint64_t f_hi, uint64_t n, uint64_t B,
               uint32_t *S_dev, uint32_t *counts_dev, const sieve_tune *tune, void *stream);

/* --- allocation-free one-shot entry point ---
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and stream behaviour as sieve_init, but the call allocates nothing: no hipMalloc,
 * hipFree or pinned host memory.  Its device scratch is one static array of 4 MiB
 * per device (held until the process ends), reached through the address
 * hipGetSymbolAddress gives for the current device at the first call on that
 * device (which also creates the library's host-side bookkeeping for it).
 * Limits: B < 2^20 and below the default medium bound 2^tile_log2 (tile_log2 = l
 * clamped to [15, 20]), so that every sieving prime stays in LDS and no bucket
 * storage is needed, and n*2^l <= 2^33 bits (one tile launch).  Requests beyond
 * these return SIEVE_E_SCRATCH before anything is enqueued.
 * Every call on one device shares that device's array (the patterns built by one
 * call are reused by the next): calls that overlap on one device race, so callers
 * order them (one stream, or events).  Device-side invariant flags of these calls
 * are not reported (sieve_check_device_errors takes an explicit context). */
int sieve_init_noalloc(uint32_t l, uint64_t f, uint64_t n, uint64_t B,
                       uint32_t *S_dev, uint32_t *counts_dev, void *stream);

/* --- helpers --- */
/* isqrt(v) for the interval (l, f, n): the bound that makes S an exact prime table
 * (Section 1.4: sieving with the primes up to sqrt(v) leaves exactly the primes). */
int sieve_required_bound(uint32_t l, uint64_t f, uint64_t n, uint64_t *B);
const char *sieve_strerror(int status);
/* The last hipError_t seen by the library on this thread (0 if none). */
int sieve_last_hip_error(void);
/* Synchronises the context's stream and reports SIEVE_E_DEVICE if a kernel
 * flagged a violated invariant since the last check (the flag is then cleared). */
int sieve_check_device_errors(sieve_ctx *ctx);

/* --- measurement ---
 * When enabled, the context records a HIP event pair around every kernel it
 * launches, on the stream it launches on, and accumulates the elapsed time per
 * kernel name.  sieve_kernel_times synchronises and copies up to cap entries:
 * names[i] (NUL-terminated, 47 chars max) and total milliseconds / launch counts. */
int sieve_ctx_set_timing(sieve_ctx *ctx, int enable);
int sieve_ctx_kernel_times(sieve_ctx *ctx, char (*names)[48], double *total_ms,
                           uint64_t *launches, uint32_t cap, uint32_t *count);
/* The default context used by sieve_init (created on first use). */
sieve_ctx *sieve_default_ctx(void);
/* Plain device copy of nbytes (multiple of 16) used to calibrate traffic counters. */
int sieve_copy_calibration(const void *src_dev, void *dst_dev, uint64_t nbytes, void *stream);

/* --- unit microbenchmarks ---
 * The measured rates the roofline figures are set against.  Runs one kernel of the
 * given kind on stream in the calling thread's default context, SYNCHRONISES, and
 * stores in *ops_per_s the operations per second of the whole device, timed with a
 * HIP event pair around the launch.  rounds (1 .. 2^20) sets the length:
 *   SIEVE_MB_LDS_OR_RANDOM  ds_or_b32 of 1024-lane workgroups (one per CU at a time)
 *                           into random words of a 2^20-bit LDS array, the access
 *                           pattern of the tile kernel's marks; 16 per lane per round
 *   SIEVE_MB_LDS_OR_SPREAD  the same with the lanes of a half wave on 32 different
 *                           banks (no bank conflicts)
 *   SIEVE_MB_VALU           32-bit integer adds and xors, eight independent chains per
 *                           lane, 16 per lane per round, eight waves per SIMD
 *   SIEVE_MB_MOD64          the 64-bit by 32-bit remainder of the offset computation
 *                           (Lemma 1's r), four independent chains per lane, 4 per lane
 *                           per round, eight waves per SIMD
 * Operations are counted per lane. */
enum { SIEVE_MB_LDS_OR_RANDOM = 0, SIEVE_MB_LDS_OR_SPREAD = 1, SIEVE_MB_VALU = 2, SIEVE_MB_MOD64 = 3 };
int sieve_microbench(uint32_t kind, uint32_t rounds, double *ops_per_s, void *stream);

/* --- inspection (tests) ---
 * Runs the offset and bucket-fill kernels for the first chunk of (l, f, n, B) and
 * copies the bucket layout to host memory: bin_start (nbins+1 entries) and the
 * in-bin offsets of every large-prime hit, widened to 32 bits (entries, up to cap).  A
 * bin's entries are its hits, each at least once, plus padding that repeats hits of
 * the bin: at most *pad_per_bin extra entries per bin (each workgroup's region of a
 * bin is rounded up to 64 bytes).  Returns the number of bins in *nbins, the bin width log2 in
 * *bin_log2, the number of bits covered in *chunk_bits and the number of large
 * primes in *nlarge.  Synchronises. */
int sieve_debug_buckets(uint32_t l, uint64_t f, uint64_t n, uint64_t B, const sieve_tune *tune,
                        uint32_t *bin_start_host, uint32_t bin_cap, uint32_t *entries_host,
                        uint64_t entry_cap, uint32_t *nbins, uint32_t *bin_log2,
                        uint64_t *chunk_bits, uint64_t *nlarge, uint64_t *nentries,
                        uint32_t *pad_per_bin);

#ifdef __cplusplus
}
#endif
#endif /* SIEVE_MI355X_H */
