"""Benchmark: sieved numbers per second of the segmented odd-only sieve on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch_1234]

The headline workload is the batch of 256 seeded interval requests (seed 1234,
centres log-uniform in [1e6, 1e15], widths log-uniform in [2^20, 2^30] numbers, B =
isqrt(v) each) sieved against one shared prime table.  A step is one sieve_batch
call over all 256 requests: first offsets, the large-prime bucket fill, every LDS
tile (pattern, medium primes, bucket drain, write-out with popcounts); the plain
per-interval kernel looped over the same requests is timed beside it.  A plain
workload name (interval_2p22, interval_1e12, interval_1e12_b6, interval_2p60)
makes a step one sieve_init call on that interval instead.

The printed line is one JSON object: the headline, its roofline (the dominant
kernel's algorithmic work per launch over its measured launch time), the plain
workloads with their own rooflines (the LDS-bound tile kernel at 1e12, the
HBM-bound bucket scatter at 2^60), launch latency of the small interval, the
serving replays (checked against the oracle's values) and the CPU oracle timed on
the host's cores.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline.
CUS, CLOCK_HZ = 256, 2.4e9
LDS_PEAK_OPS = CUS * CLOCK_HZ * 32          # one 32-bit access per LDS bank per clock, 32 banks per CU
HBM_PEAK = 8.0e12                           # bytes/s, published HBM3E peak
BUCKET_BYTES_PER_HIT = 8                    # the method's bucket entry (prime, offset), written once per hit
VALU_LANE_OPS = CUS * CLOCK_HZ * 64         # one wave64 32-bit VALU instruction per clock per CU
GB_TEST_PEAK = 32 * VALU_LANE_OPS           # Goldbach tests: 32 even numbers per 32-bit AND
FP64_OPS = 78.6e12 / 2                      # published fp64 vector peak, an fma counted as two flops


def marks_algorithmic(primes, u, v):
    """Bit-sets the tile kernel must perform: for every prime 17 <= p <= B, the odd
    multiples of p in [max(u, p^2), v] (the primes 3..13 come from the pattern)."""
    import numpy as np
    p = primes[primes >= 17].astype(np.float64)
    lo = np.maximum(float(u), p * p)
    # odd multiples m*p with lo <= m*p <= v: m odd in [ceil(lo/p), floor(v/p)]
    m0 = np.ceil(lo / p)
    m0 = m0 + (1 - np.mod(m0, 2))
    m1 = np.floor(v / p)
    m1 = m1 - (1 - np.mod(m1, 2))
    cnt = np.where(m1 >= m0, (m1 - m0) / 2 + 1, 0)
    return float(cnt.sum())


def marks_executed(primes, u, v, tile_log2=20, first_med=53):
    """LDS atomics the tile kernel executes at its default classes for 2^tile_log2-bit
    tiles: primes below first_med come from the write-out masks, primes from first_med
    to 2^(tile_log2-3) mark only the multiples m*p whose cofactor m is prime to 15 (the
    3-5 wheel), larger primes every odd multiple; all from max(u, p^2) to v."""
    import numpy as np
    assert v < (1 << 62)
    p = primes[primes >= first_med].astype(np.int64)
    m0 = np.maximum(-(-int(u) // p), p)                   # ceil(u / p), at least p
    m1 = int(v) // p
    wheel = p < (1 << (tile_log2 - 3))
    res = np.array([sum(1 for s in (1, 7, 11, 13, 17, 19, 23, 29) if s <= r) for r in range(30)], dtype=np.int64)
    coprime30 = lambda x: 8 * (x // 30) + res[x % 30]     # k in [1, x] with gcd(k, 30) = 1
    w = np.where(m1 >= m0, coprime30(m1) - coprime30(m0 - 1), 0)
    o0 = m0 + (1 - m0 % 2)
    o1 = m1 - (1 - m1 % 2)
    a = np.where(o1 >= o0, (o1 - o0) // 2 + 1, 0)
    return float(np.where(wheel, w, a).sum())


SPARSE_BYTES_PER_PRIME = 4                  # a sparse large prime is read once (its hit computed from it)
SPARSE_BYTES_PER_HIT = 4                    # and its hit, if any, written once as a table index
LAUNCH_BITS = 1 << 31                       # a launch window of the table


def sparse_counts(primes, l, f, n):
    """Sparse large primes of a single-window table (p at least the table length,
    at most one hit each) and how many of them hit it: the first odd multiple of p
    at or above max(u, p^2) (Lemma 1, Section 1.4) below v."""
    import numpy as np
    nb = n << l
    if nb > LAUNCH_BITS:
        return 0, 0
    p = primes[primes >= nb].astype(np.uint64)      # p < 2^32: p^2 fits 64 bits unsigned
    if p.size == 0:
        return 0, 0
    G0 = np.uint64(f << l)
    h = (p - np.uint64(1)) // np.uint64(2)
    r = G0 % p
    j = np.where(h >= r, h - r, h + (p - r))
    gsq = (p * p - np.uint64(1)) // np.uint64(2)
    j = np.where(gsq > G0 + j, gsq - G0, j)
    return int(p.size), int(np.count_nonzero(j < np.uint64(nb)))


def large_hits(primes, u, v, med_lim):
    import numpy as np
    p = primes[primes >= med_lim].astype(np.float64)
    if p.size == 0:
        return 0.0
    lo = np.maximum(float(u), p * p)
    m0 = np.ceil(lo / p)
    m0 = m0 + (1 - np.mod(m0, 2))
    m1 = np.floor(v / p)
    m1 = m1 - (1 - np.mod(m1, 2))
    return float(np.where(m1 >= m0, (m1 - m0) / 2 + 1, 0).sum())


def kernel_source_hash():
    """Hash of the library's code with comments and whitespace removed, so that a
    comment-only edit keeps the committed counter summaries valid."""
    import re
    h = hashlib.sha256()
    for rel in ("paper_1111_3297_amd/csrc/kernels.inc", "paper_1111_3297_amd/csrc/logsieve.inc",
                "paper_1111_3297_amd/csrc/sieve.hip"):
        with open(os.path.join(ROOT, rel)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, kernel):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def host_info():
    """Host cores this process may use and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def _golden(name):
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


def cpu_baseline_batch(reqs, l=20, budget_s=12.0):
    """The CPU oracle (single-threaded plain C) on the batch's requests in batch order
    until about budget_s seconds have passed; every total is checked against the
    oracle's golden for the batch."""
    from oracle import oracle as O
    O.build()
    g = _golden("batch_1234")
    t = time.perf_counter()
    numbers, done, ok = 0, 0, True
    for k, (f, n, B) in enumerate(reqs):
        tot = O.count_total(l, f, n, B)
        if g is not None and tot != g["requests"][k]["total"]:
            ok = False
        numbers += n << (l + 1)
        done += 1
        if time.perf_counter() - t >= budget_s:
            break
    dt = time.perf_counter() - t
    return {"value": numbers / dt, "unit": "numbers/s", "cores": 1, "kind": "oracle",
            "sample": "the first %d of the %d batch requests in batch order (%d numbers), %.1f s" % (done, len(reqs),
                                                                                                  numbers, dt),
            "totals_match_golden": ok if g is not None else None}


def cpu_baseline_batch_all_cores(reqs, l=20, per_proc_s=8.0, one_core_rate=None):
    """The same oracle in one process per usable host core (at most 16), the batch's
    requests dealt round-robin, as many of them as take about per_proc_s seconds per
    process at the single-core rate; timed from the first start to the last end."""
    import subprocess
    procs = max(1, min(16, host_info()["usable_cores"] or 1))
    rate = one_core_rate or 5e8
    want = rate * per_proc_s * procs
    take, acc = [], 0
    for r in reqs:
        take.append(r)
        acc += r[1] << (l + 1)
        if acc >= want:
            break
    code = ("import sys, json; sys.path.insert(0, %r); from oracle import oracle as O; "
            "js = json.loads(sys.argv[1]); print(json.dumps([O.count_total(%d, f, n, B) for (f, n, B) in js]))"
            % (ROOT, l))
    parts = [take[k::procs] for k in range(procs)]
    t = time.perf_counter()
    ps = [subprocess.Popen([sys.executable, "-c", code, json.dumps(p)], stdout=subprocess.PIPE) for p in parts]
    outs = [q.communicate()[0] for q in ps]
    wall = time.perf_counter() - t
    if any(q.returncode for q in ps):
        return None
    g = _golden("batch_1234")
    ok = None
    if g is not None:
        index = {(r["f"], r["n"], r["B"]): r["total"] for r in g["requests"]}
        ok = all(index.get(tuple(r)) == tot for p, o in zip(parts, outs) for r, tot in zip(p, json.loads(o)))
    return {"value": acc / wall, "unit": "numbers/s", "cores": procs, "kind": "oracle",
            "sample": "the first %d batch requests (%d numbers) dealt round-robin to %d processes, %.1f s"
                      % (len(take), acc, procs, wall), "totals_match_golden": ok}


def cpu_baseline_plain(l, f, n, B, budget_s=12.0):
    """The CPU oracle (single-threaded plain C) on a bounded prefix of a plain interval."""
    from oracle import oracle as O
    O.build()
    n0 = max(1, min(n, 16))
    t = time.perf_counter()
    O.count_total(l, f, n0, B)
    dt0 = time.perf_counter() - t
    ns = max(n0, min(n, int(n0 * budget_s / max(dt0, 1e-3))))
    t = time.perf_counter()
    tot = O.count_total(l, f, ns, B)
    dt = time.perf_counter() - t
    numbers = ns * (1 << (l + 1))
    return {"value": numbers / dt, "unit": "numbers/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d segments (%d numbers) of the same interval and bound, %.1f s"
                      % (ns, n, numbers, dt), "zero_bits": tot}


def roofline_lds(kernel, marks_per_launch, per_launch_ms, traffic, rates=None, executed=None, what="marks"):
    achieved = marks_per_launch / (per_launch_ms * 1e-3)
    out = {"bound": "lds", "kernel": kernel, "achieved": achieved / 1e9, "peak": LDS_PEAK_OPS / 1e9,
           "unit": "G%s/s" % what, "frac": achieved / LDS_PEAK_OPS, "traffic": traffic,
           "per_launch": {"algorithmic_" + what: marks_per_launch, "avg_ms": per_launch_ms}}
    if rates is not None:
        # against the measured conflict-free LDS atomic rate, and the executed atomics
        # (wheel and masks leave about half the marks out) against the random-address rate
        out["frac_of_measured_conflict_free_lds"] = achieved / rates["lds_or_spread_per_s"]
        if executed is not None:
            out["executed_marks"] = executed
            out["executed_frac_of_measured_random_lds"] = executed / (per_launch_ms * 1e-3) / rates["lds_or_random_per_s"]
    return out


def roofline_hbm(kernel, bytes_per_launch, per_launch_ms, traffic, what):
    achieved = bytes_per_launch / (per_launch_ms * 1e-3)
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": traffic,
            "per_launch": {"algorithmic_bytes": bytes_per_launch, "avg_ms": per_launch_ms, "what": what}}


def _kernel_times(ctx, fn, steps):
    """Per-kernel milliseconds per step over `steps` calls, with an event pair around
    every launch (on the stream it is launched on)."""
    import torch
    ctx.kernel_times()
    ctx.set_timing(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    return {k: {"total_ms": ms / steps, "launches_per_step": nl / steps} for k, (ms, nl) in kt.items()}


def _step_times(fn, steps, stream):
    """Milliseconds of each call, one event pair per call and nothing else."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) for a, b in ev], wall


def _pct(xs, q):
    ys = sorted(xs)
    return ys[min(len(ys) - 1, max(0, int(math.ceil(q * len(ys))) - 1))]


def run_plain(name, steps, warmup, check=True):
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, workloads
    l, f, n, B = workloads.plain_configs()[name]
    u, v = workloads.interval(l, f, n)
    S, c = api.alloc(l, n)
    ctx = api.Context.default()
    stream = torch.cuda.current_stream()
    call = lambda: api.sieve_init(l, f, n, B, S, c)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    lat, wall = _step_times(call, steps, stream)
    kernels = _kernel_times(ctx, call, steps)
    step_ms = sum(lat) / len(lat)
    out = {"name": name, "l": l, "f": f, "n": n, "B": B, "u": u, "v": v,
           "ms_per_step": step_ms, "wall_ms_per_step": 1e3 * wall / steps,
           "numbers_per_s": (v - u + 1) / (step_ms * 1e-3), "p50_ms": _pct(lat, 0.5), "p99_ms": _pct(lat, 0.99),
           "kernels": kernels}
    if check:
        g = _golden(name)
        if g is not None:
            Sh = S.cpu().numpy().view(np.uint32)
            ch = c.cpu().numpy().view(np.uint32)
            out["bit_exact"] = bool(hashlib.sha256(Sh.tobytes()).hexdigest() == g["S_sha256"]
                                    and [int(x) for x in ch] == g["counts"])
        elif name == "interval_2p22":
            out["bit_exact"] = int(c.cpu().numpy().view(np.uint32).astype(np.int64).sum()) + 1 == 295947
        else:
            out["bit_exact"] = None
    ctx.check_device_errors()
    pr = api.Primes(B)
    out["_primes"] = pr.to_tensor().cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    pr.close()
    return out


def run_latency(steps):
    """Launch latency of the small interval (1 .. 2^22, primes <= 2048): each call
    alone, waited for; device time (event pair) and host time (call to completion)."""
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, workloads
    l, f, n, B = workloads.plain_configs()["interval_2p22"]
    S, c = api.alloc(l, n)
    stream = torch.cuda.current_stream()
    for _ in range(20):
        api.sieve_init(l, f, n, B, S, c)
    torch.cuda.synchronize()
    dev, host = [], []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(steps):
        t = time.perf_counter()
        a.record(stream)
        api.sieve_init(l, f, n, B, S, c)
        b.record(stream)
        b.synchronize()
        host.append(1e3 * (time.perf_counter() - t))
        dev.append(a.elapsed_time(b))
    ok = int(c.cpu().numpy().view(np.uint32).astype(np.int64).sum()) + 1 == 295947
    return {"workload": "interval_2p22: l=15 f=0 n=64 B=2048 (sieves 1..2^22)", "calls": steps,
            "device_p50_ms": _pct(dev, 0.5), "device_p99_ms": _pct(dev, 0.99),
            "host_p50_ms": _pct(host, 0.5), "host_p99_ms": _pct(host, 0.99), "pi_2p22_ok": ok}


BATCH_WORKLOAD = ("batch_1234: 256 interval requests, seed 1234, centres log-uniform in [1e6, 1e15], widths "
                  "log-uniform in [2^20, 2^30] numbers in whole 2^21-number blocks (l=20), B = isqrt(v) each, one "
                  "shared prime table up to isqrt(max v)")


def batch_requests(l=20):
    from paper_1111_3297_amd import workloads
    reqs = []
    for f21, n21 in workloads.batch_requests(1234, 256):
        u, v = workloads.interval(l, f21, n21)
        reqs.append((f21, n21, math.isqrt(v)))
    return reqs


def run_batch(steps, warmup, log, loops=2):
    """The 256-request batch: one persistent batched launch per step, against looping
    the plain per-interval sieve over the same requests."""
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, autotune
    l = 20
    reqs = batch_requests(l)
    numbers = sum(n << (l + 1) for (_, n, _) in reqs)
    pr = api.Primes(max(B for (_, _, B) in reqs))
    outs = []
    for (f, n, B) in reqs:
        S, c = api.alloc(l, n)
        outs.append((f, n, B, S, c))
    ctx = api.Context()
    t = time.perf_counter()
    tune = autotune.tune_batch(pr, l, outs, ctx=ctx, log=log)
    tune_s = time.perf_counter() - t
    stream = torch.cuda.current_stream()
    call = lambda: ctx.batch(pr, l, outs, tune=tune)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    lat, wall = _step_times(call, steps, stream)
    kernels = _kernel_times(ctx, call, max(2, steps // 4))
    ms = sum(lat) / len(lat)
    bit_exact = None
    g = _golden("batch_1234")
    if g is not None:
        bit_exact = True
        for (f, n, B, S, c), r in zip(outs, g["requests"]):
            ch = c.cpu().numpy().view(np.uint32)
            if hashlib.sha256(ch.astype("<u4").tobytes()).hexdigest() != r["counts_sha256"] or \
                    hashlib.sha256(S.cpu().numpy().tobytes()).hexdigest() != r["S_sha256"]:
                bit_exact = False
                break

    def plain_loop():
        for (f, n, B, S, c) in outs:
            ctx.sieve(l, f, n, B, S, c, primes=pr)

    def init_loop():
        for (f, n, B, S, c) in outs:
            api.sieve_init(l, f, n, B, S, c)

    plain_loop()
    pl, _ = _step_times(plain_loop, loops, stream)
    init_loop()
    il, _ = _step_times(init_loop, 1, stream)
    ctx.check_device_errors()
    ms_loop, ms_init = sum(pl) / len(pl), sum(il) / len(il)
    primes = pr.to_tensor().cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    return {"reqs": reqs, "numbers": numbers, "tune": tune, "autotune_s": round(tune_s, 2), "ms_per_step": ms,
            "wall_ms_per_step": 1e3 * wall / steps, "numbers_per_s": numbers / (ms * 1e-3),
            "p50_ms": _pct(lat, 0.5), "p99_ms": _pct(lat, 0.99), "kernels": kernels, "bit_exact": bit_exact,
            "plain_loop_shared_table": {"ms": ms_loop, "numbers_per_s": numbers / (ms_loop * 1e-3)},
            "plain_loop_sieve_init": {"ms": ms_init, "numbers_per_s": numbers / (ms_init * 1e-3)},
            "speedup_vs_plain_loop": ms_loop / ms, "_primes": primes}


def batch_work(primes, reqs, tune, l=20):
    """Algorithmic marks (every prime 17 <= p <= B_i) and large-prime hits (primes at or
    above the tuned medium bound) summed over the batch's requests."""
    import numpy as np
    med = 1 << int(tune.get("medium_log2") or tune.get("tile_log2") or 20)
    marks = hits = 0.0
    for (f, n, B) in reqs:
        u, v = f * (1 << (l + 1)) + 1, (f + n) * (1 << (l + 1))
        P = primes[: int(np.searchsorted(primes, B, side="right"))]
        marks += marks_algorithmic(P, u, v)
        hits += large_hits(P, u, v, med)
    return marks, hits


def serving_check(res, g):
    """Every served request's zero-bit total and counts digest against the oracle's."""
    import numpy as np
    if g is None:
        return None
    for rid, r in res.items():
        c = r["counts"]
        want = g["requests"][rid]
        if int(c.astype(np.int64).sum()) != want[0] or \
                hashlib.sha256(c.astype("<u4").tobytes()).hexdigest()[:16] != want[1]:
            return False
    return True


def run_serving(seconds, speedups, tune, log, slots=3):
    """Open-loop replays of the seeded Poisson stream (seed 99, 200 requests/s for 60 s,
    90% as in the batch workload, 10% of width 2^28 centred in [1e16, 2^62]), 64 GB
    budget: continuous batching against a first-come-first-served plain-kernel
    server, at the stated rate over `seconds` and time-compressed by each speedup.
    Every served request's counts are checked against the oracle's golden values."""
    from paper_1111_3297_amd import api, serve
    l = 20
    g = _golden("serve_99")
    base = serve.serving_requests(l=l, limit_s=seconds)
    pr = api.Primes(max(r.B for r in base))
    ex = serve.GpuExecutor(pr, l, slots=slots, tune=tune)
    ex0 = serve.PlainExecutor(pr, l)
    # both servers first replay the opening half second untimed (allocator and pinned
    # host memory warm-up), so that neither pays it inside its measured replay
    warm = [r for r in base if r.arrival < 0.5]
    serve.Server(ex, l=l, budget_bytes=64 << 30).run(warm)
    serve.Server(ex0, l=l, budget_bytes=64 << 30, max_group=1).run(warm)
    keep = ("requests", "numbers", "span_s", "numbers_per_s", "p50_ms", "p99_ms", "max_ms", "peak_bytes")
    out = {"workload": "Poisson stream seed 99, 200 req/s for %g s (12040 requests over the full 60 s), 90%% as the "
                       "batch, 10%% width 2^28 centred in [1e16, 2^62], B = isqrt(v), 64 GB budget" % seconds,
           "slots": slots, "replays": []}
    for sp in [1.0] + list(speedups):
        reqs = base if sp == 1.0 else serve.serving_requests(l=l, limit_s=seconds, speedup=sp)
        rec = {"speedup": sp, "offered_req_per_s": 200.0 * sp}
        for name, exe, mg in (("continuous_batching", ex, 64), ("plain_fcfs", ex0, 1)):
            prog = (lambda now, done, tot, name=name, sp=sp: log("serving x%g %s: %.0f s, %d of %d done"
                                                                  % (sp, name, now, done, tot)))
            res, st = serve.Server(exe, l=l, budget_bytes=64 << 30, max_group=mg, progress=prog).run(reqs)
            rec[name] = {k: st[k] for k in keep}
            rec[name]["bit_exact_counts"] = serving_check(res, g)
            log("serving x%g %s: p50 %.3f ms p99 %.3f ms, %.3g numbers/s" % (sp, name, st["p50_ms"], st["p99_ms"],
                                                                            st["numbers_per_s"]))
        out["replays"].append(rec)
    return out


def run_goldbach(steps, Q=1 << 16):
    """The Goldbach check of every even number of the 1e12 table (2^32 numbers,
    u+1 .. v) against the odd primes q <= Q: the table from sieve_init (checked against
    the oracle's golden), then sieve_goldbach timed alone; two segments recomputed by
    the oracle."""
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, workloads
    l, f, n, B = workloads.plain_configs()["interval_1e12"]
    S, c = api.alloc(l, n)
    api.sieve_init(l, f, n, B, S, c)
    ctx = api.Context()
    pr = api.Primes(max(B, Q))
    torch.cuda.synchronize()
    g = _golden("interval_1e12")
    table_ok = g is not None and hashlib.sha256(S.cpu().numpy().tobytes()).hexdigest() == g["S_sha256"]
    stream = torch.cuda.current_stream()
    outs = {}

    def call():
        outs["r"] = ctx.goldbach(pr, l, f, n, S, Q)
    for _ in range(3):
        call()
    lat, _ = _step_times(call, steps, stream)
    kernels = _kernel_times(ctx, call, max(2, steps // 2))
    maxq, argk, fails, _ = outs["r"]
    mh, ah, fh = maxq.cpu().numpy().view(np.uint32), argk.cpu().numpy().view(np.uint64), fails.cpu().numpy()
    from oracle import oracle as O
    ok = True
    idx = []
    Ptab = O.odd_primes(Q)
    for t in (1, n - 1):
        So, _ = O.sieve(l, f + t - 1, 2, B)
        mq, mx, ak, fl = O.goldbach(l, f + t - 1, 2, So, Q)
        ok = ok and (int(mh[t]), int(ah[t]), int(fh[t])) == (int(mx[1]), int(ak[1]) + ((t - 1) << l), int(fl[1]))
        seg = mq[1 << l:]
        idx.append(float((np.searchsorted(Ptab, seg[seg > 0]) + 1).mean()))
    tests = float(np.mean(idx)) * (n << l)
    kt = kernels["k_goldbach"]
    per_ms = kt["total_ms"] / kt["launches_per_step"]
    nb = (n << l) // 8 + 16 * n
    u, v = workloads.interval(l, f, n)
    best = int(np.argmax(mh))
    return {"workload": "Goldbach check of the even numbers %d .. %d (2^32 numbers) against the table of "
                        "interval_1e12 and the odd primes q <= %d" % (u + 1, v, Q),
            "ms_per_call": sum(lat) / len(lat), "p99_ms": _pct(lat, 0.99),
            "even_numbers_per_s": (n << l) / (sum(lat) / len(lat) * 1e-3),
            "largest_least_q": int(mh[best]), "at_N": int(u + 1 + 2 * int(ah[best])), "failures": int(fh.sum()),
            "table_bit_exact": table_ok, "sampled_segments_bit_exact": ok,
            "kernels_ms_per_call": {k: round(x["total_ms"], 4) for k, x in kernels.items()},
            "roofline": roofline_hbm("k_goldbach", nb, per_ms, traffic_from_profile("goldbach_1e12", "k_goldbach"),
                                     "the table read once (%d bytes) and 16 bytes of output per segment" % ((n << l) // 8)),
            "roofline_alu": {"bound": "alu", "kernel": "k_goldbach", "unit": "Gtests/s",
                             "achieved": tests / (per_ms * 1e-3) / 1e9, "peak": GB_TEST_PEAK / 1e9,
                             "frac": tests / (per_ms * 1e-3) / GB_TEST_PEAK,
                             "per_launch": {"tests": tests, "avg_ms": per_ms,
                                            "what": "(number, prime) tests in ascending q up to each number's least q "
                                                    "(mean index %.2f from two oracle segments), 32 per 32-bit lane "
                                                    "operation at the peak" % float(np.mean(idx))}}}


def log_adds(primes, u, v):
    """Additions the log-add sieve must make: every odd multiple m p (m >= 1) of every
    odd prime p of the factor base in [u, v]."""
    import numpy as np
    p = primes.astype(np.int64)
    hi = (int(v) // p + 1) // 2            # odd multiples <= v
    lo = ((int(u) - 1) // p + 1) // 2      # odd multiples <= u - 1
    return float((hi - lo).sum())


def run_logsieve(steps, B=1 << 20, T=34):
    """The log-add sieve of the 1e12 interval (2^32 odd numbers) with the odd primes
    up to B as factor base and threshold T: candidates table and counts, timed per
    call; two segments recomputed by the oracle."""
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, workloads
    l, f, n, _ = workloads.plain_configs()["interval_1e12"]
    u, v = workloads.interval(l, f, n)
    C, c = api.alloc(l, n)
    ctx = api.Context()
    pr = api.Primes(B)
    stream = torch.cuda.current_stream()
    call = lambda: ctx.logsieve(l, f, n, B, T, C, c, primes=pr)
    for _ in range(2):
        call()
    lat, _ = _step_times(call, steps, stream)
    kernels = _kernel_times(ctx, call, max(2, steps // 2))
    ctx.check_device_errors()
    Ch, ch = C.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32)
    from oracle import oracle as O
    ok = True
    w = 1 << (l - 5)
    for t in (0, n - 1):
        Co, co, _ = O.logsieve(l, f + t, 1, B, T, with_sums=False)
        ok = ok and bool(np.array_equal(Ch[t * w:(t + 1) * w], Co)) and int(ch[t]) == int(co[0])
    primes = pr.to_tensor().cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    adds = log_adds(primes, u, v)
    kt = kernels["k_logtile"]
    per_ms = kt["total_ms"] / kt["launches_per_step"]
    ms = sum(lat) / len(lat)
    return {"workload": "log-add sieve of the odd numbers %d .. %d (2^32 positions) by the odd primes <= %d, "
                        "threshold %d" % (u, v, B, T),
            "ms_per_call": ms, "p99_ms": _pct(lat, 0.99), "numbers_per_s": (v - u + 1) / (ms * 1e-3),
            "candidates": int(ch.astype(np.int64).sum()), "sampled_segments_bit_exact": ok,
            "kernels_ms_per_call": {k: round(x["total_ms"], 4) for k, x in kernels.items()},
            "roofline": dict(roofline_lds("k_logtile", adds / kt["launches_per_step"], per_ms,
                                          traffic_from_profile("logsieve_1e12", "k_logtile"), what="adds"),
                             note="an LDS add of floor(log2 p) at every odd multiple of every factor-base prime "
                                  "(%.4g per call)" % adds)}


def _probable_prime(N):
    """Miller-Rabin to the first twelve prime bases (deterministic below 3.1e23)."""
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if N % p == 0:
            return N == p
    d, s = N - 1, 0
    while d % 2 == 0:
        d, s = d // 2, s + 1
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


def run_wide(steps, l=20, f=2**49, n=1024):
    """The prime table of 2^30 odd numbers from 2^70 + 1 (beyond 2^64: a 128-bit
    start, sieving primes up to isqrt(v) = 2^35, i.e. above 32 bits), timed per call;
    600 sampled bits checked against Miller-Rabin (zero bit <=> prime)."""
    import random
    import numpy as np
    import torch
    from paper_1111_3297_amd import api
    u, v = f * 2**(l + 1) + 1, (f + n) * 2**(l + 1)
    B = math.isqrt(v)
    S, c = api.alloc(l, n)
    ctx = api.Context()
    stream = torch.cuda.current_stream()
    call = lambda: ctx.wide(l, f, n, B, S, c)
    for _ in range(2):
        call()
    lat, _ = _step_times(call, steps, stream)
    kernels = _kernel_times(ctx, call, max(2, steps // 2))
    ctx.check_device_errors()
    Sh, ch = S.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32)
    rng = random.Random(70)
    ok = True
    for j in [rng.randrange(n << l) for _ in range(600)]:
        ok = ok and (((int(Sh[j >> 5]) >> (j & 31)) & 1) == (0 if _probable_prime(u + 2 * j) else 1))
    ms = sum(lat) / len(lat)
    # remainders the method takes: one per prime above 2^32 up to B (Lemma 1's first
    # offset), B = 2^35 here, pi(2^35) - pi(2^32) by the published values (OEIS
    # A007053); each needs at least the Horner steps of a 128-bit start of this size
    # (the top 52 bits, then 17-bit digits) at four fp64 operations per step, plus the
    # reciprocal: the fp64 peak 78.6 TFLOP/s counts an fma as two, so 39.3e12
    # operations per second
    assert B == 2**35
    nrem = 1480206279 - 203280221
    steps = 1 + max(0, -(-((f << l).bit_length() - 52) // 17))
    ops = 4 * steps + 1
    kw = kernels["k_wide_hits"]
    peak = FP64_OPS / ops
    roof = {"bound": "alu", "kernel": "k_wide_hits", "unit": "Gremainders/s",
            "achieved": nrem / (kw["total_ms"] * 1e-3) / 1e9, "peak": peak / 1e9,
            "frac": nrem / (kw["total_ms"] * 1e-3) / peak,
            "per_call": {"remainders": nrem, "ms": kw["total_ms"], "launches": kw["launches_per_step"],
                         "what": "one 128-bit remainder per prime in (2^32, B] (%d fp64 operations each at "
                                 "the peak), plus its hit listed for the sort by table range (k_hits_sort and "
                                 "k_sparse_apply, timed apart) or OR-ed into the table" % ops}}
    return {"workload": "prime table of the odd numbers 2^70 + 1 .. 2^70 + 2^31 (2^30 bits) with the odd "
                        "primes up to %d (128-bit start, sieving primes above 32 bits)" % B,
            "ms_per_call": ms, "p99_ms": _pct(lat, 0.99), "numbers_per_s": (v - u + 1) / (ms * 1e-3),
            "primes": int(ch.astype(np.int64).sum()), "sampled_bits_match_miller_rabin": ok,
            "kernels_ms_per_call": {k: round(x["total_ms"], 4) for k, x in kernels.items()},
            "launches_per_call": {k: x["launches_per_step"] for k, x in kernels.items()},
            "roofline": roof}


def unit_rates():
    """Measured unit rates the roofline figures are set against: the library's LDS-atomic, VALU
    and 64-bit remainder microbenchmarks (sieve_microbench, median of three) and its plain HBM
    copy of 1 GiB."""
    import ctypes
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, _lib
    rates = {}
    for kind, rounds in (("lds_or_random", 2048), ("lds_or_spread", 2048), ("valu_int32", 16384), ("mod64", 1024)):
        api.microbench(kind, 64)                                  # warm-up
        rates[kind + "_per_s"] = float(np.median([api.microbench(kind, rounds) for _ in range(3)]))
    nb = 1 << 30
    a = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    copy = lambda: _lib.check(_lib.load().sieve_copy_calibration(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                                                  nb, ctypes.c_void_p(st.cuda_stream)), "sieve_copy_calibration")
    copy()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(5):
        copy()
    e1.record(st)
    e1.synchronize()
    rates["hbm_copy_bytes_per_s"] = 5 * 2.0 * nb / (e0.elapsed_time(e1) * 1e-3)   # bytes read + written
    del a, b
    clk_cu = CLOCK_HZ * CUS
    rates["per_clock_per_cu"] = {"lds_or_random": rates["lds_or_random_per_s"] / clk_cu,
                                 "lds_or_spread": rates["lds_or_spread_per_s"] / clk_cu,
                                 "valu_int32": rates["valu_int32_per_s"] / clk_cu}
    return rates


def plain_rooflines(rec, rates):
    """The roofline of a plain workload's dominant kernel: the tile kernel by LDS marks,
    or the bucket scatter by the method's bucket bytes."""
    primes = rec.pop("_primes")
    u, v = rec["u"], rec["v"]
    ks = rec["kernels"]
    dom = max(ks, key=lambda k: ks[k]["total_ms"])
    out = {}
    if "k_bucket_scatter" in ks:
        # the bucketed primes: from the medium bound on, up to the sparse ones when
        # those take their own path (p at least the table length)
        bucketed = primes[primes < (rec["n"] << rec["l"])] if "k_sparse_collect" in ks else primes
        hits = large_hits(bucketed, u, v, 1 << 20)
        kt = ks["k_bucket_scatter"]
        per_ms = kt["total_ms"] / kt["launches_per_step"]
        out["k_bucket_scatter"] = roofline_hbm("k_bucket_scatter", BUCKET_BYTES_PER_HIT * hits / kt["launches_per_step"],
                                               per_ms, traffic_from_profile(rec["name"], "k_bucket_scatter"),
                                               "%d bytes per large-prime hit (%.4g hits per step)"
                                               % (BUCKET_BYTES_PER_HIT, hits))
    if "k_sparse_collect" in ks:
        nsp, hits = sparse_counts(primes, rec["l"], rec["f"], rec["n"])
        kt = ks["k_sparse_collect"]
        per_ms = kt["total_ms"] / kt["launches_per_step"]
        out["k_sparse_collect"] = roofline_hbm(
            "k_sparse_collect", (SPARSE_BYTES_PER_PRIME * nsp + SPARSE_BYTES_PER_HIT * hits) / kt["launches_per_step"],
            per_ms, traffic_from_profile(rec["name"], "k_sparse_collect"),
            "%d bytes per sparse large prime (%d) and %d per hit (%d)"
            % (SPARSE_BYTES_PER_PRIME, nsp, SPARSE_BYTES_PER_HIT, hits))
    kt = ks.get("k_tile")
    if kt:
        per_ms = kt["total_ms"] / kt["launches_per_step"]
        marks = marks_algorithmic(primes, u, v) / kt["launches_per_step"]
        ex = marks_executed(primes, u, v) / kt["launches_per_step"] if rec["l"] == 20 and rates else None
        out["k_tile"] = roofline_lds("k_tile", marks, per_ms, traffic_from_profile(rec["name"], "k_tile"), rates, ex)
    rec["dominant_kernel"] = dom
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch_1234", help="batch_1234 (headline) or a plain interval workload")
    ap.add_argument("--also", default="interval_1e12,interval_2p60,serve_req6388",
                    help="comma list of plain workloads to report")
    ap.add_argument("--latency-steps", type=int, default=200, help="calls of the small interval for launch latency")
    ap.add_argument("--goldbach-steps", type=int, default=10, help="timed Goldbach checks of the 1e12 table (0: skip)")
    ap.add_argument("--logsieve-steps", type=int, default=10, help="timed log-add sieves of the 1e12 interval (0: skip)")
    ap.add_argument("--wide-steps", type=int, default=5, help="timed prime tables at 2^70 (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="seconds of the request stream to replay (0: skip)")
    ap.add_argument("--serve-speedups", default="10,30,100", help="time-compressed replays of the same stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-unit-rates", action="store_true", help="skip the LDS / VALU / copy microbenchmarks")
    ap.add_argument("--unit-rates-only", action="store_true", help="only run the microbenchmarks and print their rates")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run the library's plain copy kernel over this many bytes, 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(a sharded run would split each interval into contiguous segment ranges, or route whole "
              "requests, one GPU each); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        from paper_1111_3297_amd import _lib
        import ctypes
        nb = args.copy_calibration - args.copy_calibration % 16
        a = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            _lib.check(_lib.load().sieve_copy_calibration(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                                          nb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
                       "sieve_copy_calibration")
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "launches": 5}))
        return
    if args.unit_rates_only:
        print(json.dumps({"unit_rates": unit_rates()}), flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    rates = None if args.no_unit_rates else unit_rates()
    out = {"metric": "sieved numbers/sec at 1 GPU (batched vs plain, bit-exact); p99 latency", "unit": "numbers/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic"}
    tune = None
    if args.workload == "batch_1234":
        log("batch: autotune and %d timed steps" % args.steps)
        rec = run_batch(args.steps, args.warmup, log)
        primes = rec.pop("_primes")
        tune = rec["tune"]
        marks, hits = batch_work(primes, rec["reqs"], tune)
        ks = rec["kernels"]
        dom = max(ks, key=lambda k: ks[k]["total_ms"])
        kt = ks[dom]
        per_ms = kt["total_ms"] / kt["launches_per_step"]
        if dom == "k_bucket_scatter":
            roof = roofline_hbm(dom, BUCKET_BYTES_PER_HIT * hits / kt["launches_per_step"], per_ms,
                                traffic_from_profile("batch_1234", dom),
                                "%d bytes per large-prime hit (%.4g hits per step)" % (BUCKET_BYTES_PER_HIT, hits))
        else:
            roof = roofline_lds(dom, marks / kt["launches_per_step"], per_ms, traffic_from_profile("batch_1234", dom),
                                rates)
        out.update({"value": rec["numbers_per_s"], "ms_per_step": rec["ms_per_step"],
                    "config": {"workload": BATCH_WORKLOAD,
                               "mode": "one sieve_batch of all 256 requests per step (tuned %s); the plain "
                                       "per-interval kernel looped over the same requests beside it" % (tune,),
                               "numbers_per_step": rec["numbers"]},
                    "p50_ms": rec["p50_ms"], "p99_ms": rec["p99_ms"], "wall_ms_per_step": rec["wall_ms_per_step"],
                    "bit_exact": rec["bit_exact"],
                    "plain": {"loop_shared_table": rec["plain_loop_shared_table"],
                              "loop_sieve_init": rec["plain_loop_sieve_init"],
                              "batched_speedup_vs_loop": rec["speedup_vs_plain_loop"]},
                    "roofline": roof, "autotune_s": rec["autotune_s"],
                    "work_per_step": {"algorithmic_marks": marks, "large_prime_hits": hits},
                    "kernels_ms_per_step": {k: round(x["total_ms"], 4) for k, x in ks.items()}})
        headline_reqs = rec["reqs"]
    else:
        rec = run_plain(args.workload, args.steps, args.warmup)
        roofs = plain_rooflines(rec, rates)
        dom = rec["dominant_kernel"]
        out.update({"value": rec["numbers_per_s"], "ms_per_step": rec["ms_per_step"],
                    "config": {"workload": "%s: l=%d f=%d n=%d B=%d (u=%d, v=%d)" % (
                        args.workload, rec["l"], rec["f"], rec["n"], rec["B"], rec["u"], rec["v"]),
                        "mode": "plain (one sieve_init per step, prime generation included)"},
                    "p50_ms": rec["p50_ms"], "p99_ms": rec["p99_ms"], "bit_exact": rec.get("bit_exact"),
                    "roofline": roofs.get(dom) or next(iter(roofs.values()), None),
                    "kernels_ms_per_step": {k: round(x["total_ms"], 4) for k, x in rec["kernels"].items()}})
        headline_reqs = None
    also, rooflines = {}, []
    for name in [x for x in args.also.split(",") if x and x != "none" and x != args.workload]:
        log("plain workload %s" % name)
        r = run_plain(name, max(3, args.steps // 2), 2)
        roofs = plain_rooflines(r, rates)
        for k, ro in roofs.items():
            rooflines.append(dict(ro, workload=name))
        also[name] = {kk: r[kk] for kk in ("numbers_per_s", "ms_per_step", "p50_ms", "p99_ms", "bit_exact", "B",
                                          "dominant_kernel")}
        also[name]["kernels_ms_per_step"] = {kk: round(x["total_ms"], 4) for kk, x in r["kernels"].items()}
    if args.goldbach_steps > 0:
        log("goldbach check")
        out["goldbach"] = run_goldbach(args.goldbach_steps)
        rooflines.append(dict(out["goldbach"]["roofline"], workload="goldbach_1e12"))
    if args.logsieve_steps > 0:
        log("log-add sieve")
        out["logsieve"] = run_logsieve(args.logsieve_steps)
        rooflines.append(dict(out["logsieve"]["roofline"], workload="logsieve_1e12"))
    if args.wide_steps > 0:
        log("prime table beyond 2^64")
        out["wide"] = run_wide(args.wide_steps)
        rooflines.append(dict(out["wide"]["roofline"], workload="wide_2p70"))
    out["also"] = also
    out["rooflines"] = rooflines
    if args.latency_steps > 0:
        log("latency: %d calls of the small interval" % args.latency_steps)
        out["latency_small"] = run_latency(args.latency_steps)
    if args.serve_seconds > 0:
        sps = [float(x) for x in args.serve_speedups.split(",") if x]
        out["serving"] = run_serving(args.serve_seconds, sps, tune, log)
    if rates is not None:
        out["unit_rates"] = rates
    out["host"] = host_info()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        if headline_reqs is not None:
            cb = cpu_baseline_batch(headline_reqs)
            out["cpu_baseline"] = cb
            out["cpu_baseline_all_cores"] = cpu_baseline_batch_all_cores(headline_reqs, one_core_rate=cb["value"])
        else:
            out["cpu_baseline"] = cpu_baseline_plain(rec["l"], rec["f"], rec["n"], rec["B"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
