"""Benchmark: sieved numbers per second of the segmented odd-only sieve on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload interval_1e12]

A step is one full sieve_init call on the workload: device prime generation up to
B, first offsets, the large-prime bucket fill (when B reaches the bucket range),
every LDS tile (pattern, medium primes, bucket drain, write-out with popcounts).
Inputs are interval parameters; outputs land in HBM.  The line printed is one
JSON object.  Its roofline entry rates the tile kernel by algorithmic marks (every
odd multiple of every prime 17 <= p <= B in the interval, at or above p^2) per
second against one 32-bit LDS access per bank per clock on every CU; its
cpu_baseline entry times the plain CPU oracle on the same interval.
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
LDS_PEAK_OPS = CUS * CLOCK_HZ * 32          # one 32-bit LDS access per bank per clock, 32 banks
HBM_PEAK = 8.0e12                           # bytes/s


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
    for rel in ("paper_1111_3297_amd/csrc/kernels.inc", "paper_1111_3297_amd/csrc/sieve.hip"):
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


def cpu_baseline(l, f, n, B, budget_s=12.0):
    """The CPU oracle (single-threaded plain C) on a bounded prefix of the workload."""
    from oracle import oracle as O
    O.build()
    # calibrate on a small prefix, then run a prefix sized to the budget
    n0 = max(1, min(n, 16))
    t = time.perf_counter()
    O.count_total(l, f, n0, B)
    dt0 = time.perf_counter() - t
    ns = max(n0, min(n, int(n0 * budget_s / max(dt0, 1e-3))))
    t = time.perf_counter()
    O.count_total(l, f, ns, B)
    dt = time.perf_counter() - t
    numbers = ns * (1 << (l + 1))
    return {"value": numbers / dt, "unit": "numbers/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of %d segments (%d numbers) of the same interval and bound, %.1f s"
                      % (ns, n, numbers, dt)}


def cpu_baseline_all_cores(l, f, n, B, per_proc_s=8.0):
    """The same oracle in one process per host core (at most 16), each on its own contiguous
    range of segments of the workload, timed from the first start to the last end."""
    import subprocess
    from oracle import oracle as O
    O.build()
    procs = max(1, min(16, os.cpu_count() or 1))
    n0 = max(1, min(n, 8))
    t = time.perf_counter()
    O.count_total(l, f, n0, B)
    per_seg = max(time.perf_counter() - t, 1e-6) / n0
    each = max(1, min(n // procs, int(per_proc_s / per_seg)))
    code = ("import sys; sys.path.insert(0, %r); from oracle import oracle as O; "
            "O.count_total(%d, int(sys.argv[1]), %d, %d)" % (ROOT, l, each, B))
    t = time.perf_counter()
    ps = [subprocess.Popen([sys.executable, "-c", code, str(f + k * each)]) for k in range(procs)]
    rcs = [q.wait() for q in ps]
    wall = time.perf_counter() - t
    if any(rcs):
        return None
    numbers = procs * each * (1 << (l + 1))
    return {"value": numbers / wall, "unit": "numbers/s", "cores": procs, "kind": "oracle",
            "sample": "segments %d..%d of %d (%d numbers) of the same interval and bound, %d processes of %d "
                      "segments, %.1f s" % (0, procs * each - 1, n, numbers, procs, each, wall)}


def run_plain(name, steps, warmup, check=True):
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, workloads
    l, f, n, B = workloads.plain_configs()[name]
    u, v = workloads.interval(l, f, n)
    S, c = api.alloc(l, n)
    ctx = api.Context.default()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        api.sieve_init(l, f, n, B, S, c)
    torch.cuda.synchronize()
    # the timed steps: one event pair per step and nothing else on the stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        api.sieve_init(l, f, n, B, S, c)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = sorted(a.elapsed_time(b) for a, b in ev)
    # the same steps again with an event pair around every kernel launch (on the
    # stream it is launched on), for the per-kernel durations and the roofline
    ctx.kernel_times()                     # drop anything recorded so far
    ctx.set_timing(True)
    ek = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ek:
        a.record(stream)
        api.sieve_init(l, f, n, B, S, c)
        b.record(stream)
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    step_ms_kev = sum(a.elapsed_time(b) for a, b in ek) / steps
    step_ms = sum(lat) / len(lat)
    numbers = v - u + 1
    out = {"name": name, "l": l, "f": f, "n": n, "B": B, "u": u, "v": v,
           "ms_per_step": step_ms, "wall_ms_per_step": 1e3 * wall / steps,
           "ms_per_step_with_kernel_events": step_ms_kev,
           "numbers_per_s": numbers / (step_ms * 1e-3),
           "p50_ms": lat[len(lat) // 2], "p99_ms": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
           "kernels": {k: {"total_ms": ms / steps, "launches_per_step": nl / steps} for k, (ms, nl) in kt.items()}}
    if check:
        gpath = os.path.join(ROOT, "tests", "golden", name + ".json")
        if os.path.exists(gpath):
            with open(gpath) as fh:
                g = json.load(fh)
            Sh = S.cpu().numpy().view(np.uint32)
            ch = c.cpu().numpy().view(np.uint32)
            out["bit_exact"] = bool(hashlib.sha256(Sh.tobytes()).hexdigest() == g["S_sha256"]
                                    and [int(x) for x in ch] == g["counts"])
        else:
            out["bit_exact"] = None
    pr = api.Primes(B)
    out["_primes"] = pr.to_tensor().cpu().numpy().view(np.uint32)
    torch.cuda.synchronize()
    pr.close()
    return out


def run_batch_bench(steps, log):
    """The 256-request batch (seed 1234, B = isqrt(v) each): one persistent batched
    launch per step against looping the plain per-interval sieve."""
    import numpy as np
    import torch
    from paper_1111_3297_amd import api, autotune, workloads
    l = 20
    reqs = []
    for f21, n21 in workloads.batch_requests(1234, 256):
        u, v = workloads.interval(l, f21, n21)
        reqs.append((f21, n21, math.isqrt(v)))
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

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / k

    ms_batch = timed(lambda: ctx.batch(pr, l, outs, tune=tune), steps)
    bit_exact = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch_1234.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
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

    ms_loop = timed(plain_loop, 2)
    ms_init = timed(init_loop, 1)
    ctx.check_device_errors()
    return {"workload": "256 requests, seed 1234: centres log-uniform in [1e6, 1e15], widths log-uniform in "
                        "[2^20, 2^30] numbers in whole 2^21-number blocks, B = isqrt(v) each (l=20)",
            "numbers": numbers, "tune": tune, "autotune_s": round(tune_s, 2),
            "batched": {"ms": ms_batch, "numbers_per_s": numbers / (ms_batch * 1e-3)},
            "plain_loop_shared_table": {"ms": ms_loop, "numbers_per_s": numbers / (ms_loop * 1e-3)},
            "plain_loop_sieve_init": {"ms": ms_init, "numbers_per_s": numbers / (ms_init * 1e-3)},
            "speedup_vs_plain_loop": ms_loop / ms_batch, "bit_exact": bit_exact}


def run_serving_bench(seconds, tune, slots=3):
    """Open-loop replay of the seeded Poisson stream (seed 99, 200 requests/s,
    90% as in the batch workload, 10% of width 2^28 centred in [1e16, 2^62]) for the
    first `seconds` seconds, 64 GB budget: continuous batching against a first come
    first served plain-kernel server."""
    from paper_1111_3297_amd import api, serve
    l = 20
    reqs = serve.serving_requests(l=l, limit_s=seconds)
    pr = api.Primes(max(r.B for r in reqs))
    ex = serve.GpuExecutor(pr, l, slots=slots, tune=tune)
    ex0 = serve.PlainExecutor(pr, l)
    # both servers first replay the opening half second untimed (allocator and pinned
    # host memory warm-up), so that neither pays it inside its measured replay
    warm = [r for r in reqs if r.arrival < 0.5]
    serve.Server(ex, l=l, budget_bytes=64 << 30).run(warm)
    serve.Server(ex0, l=l, budget_bytes=64 << 30, max_group=1).run(warm)
    _, st = serve.Server(ex, l=l, budget_bytes=64 << 30).run(reqs)
    _, st0 = serve.Server(ex0, l=l, budget_bytes=64 << 30, max_group=1).run(reqs)
    keep = ("requests", "numbers", "span_s", "numbers_per_s", "p50_ms", "p99_ms", "max_ms", "peak_bytes")
    return {"workload": "Poisson stream seed 99, 200 req/s, first %g s of 60 s, B = isqrt(v), 64 GB budget" % seconds,
            "continuous_batching": {k: st[k] for k in keep},
            "plain_fcfs": {k: st0[k] for k in keep}}


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
    clk_cu = 2.4e9 * 256
    rates["per_clock_per_cu"] = {"lds_or_random": rates["lds_or_random_per_s"] / clk_cu,
                                 "lds_or_spread": rates["lds_or_spread_per_s"] / clk_cu,
                                 "valu_int32": rates["valu_int32_per_s"] / clk_cu}
    return rates


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="interval_1e12")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--also", default="interval_2p60", help="comma list of extra plain workloads to report")
    ap.add_argument("--batch-steps", type=int, default=5, help="timed batched launches (0: skip the batch bench)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="seconds of the request stream to replay (0: skip)")
    ap.add_argument("--no-unit-rates", action="store_true", help="skip the LDS / VALU / copy microbenchmarks")
    ap.add_argument("--unit-rates-only", action="store_true", help="only run the microbenchmarks and print their rates")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run the library's plain copy kernel over this many bytes, 5 times (counter calibration)")
    args = ap.parse_args()
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
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(a sharded run would split the interval into contiguous segment ranges, one per GPU); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    main_rec = run_plain(args.workload, args.steps, args.warmup)
    primes = main_rec.pop("_primes")
    u, v = main_rec["u"], main_rec["v"]
    marks = marks_algorithmic(primes, u, v)
    kt = main_rec["kernels"].get("k_tile", {"total_ms": float("nan"), "launches_per_step": 1})
    per_launch_ms = kt["total_ms"] / kt["launches_per_step"]
    marks_per_launch = marks / kt["launches_per_step"]
    achieved = marks_per_launch / (per_launch_ms * 1e-3)
    traffic = traffic_from_profile(args.workload, "k_tile")
    roof = {"bound": "lds", "kernel": "k_tile", "achieved": achieved / 1e9, "peak": LDS_PEAK_OPS / 1e9,
            "unit": "Gmarks/s", "frac": achieved / LDS_PEAK_OPS, "traffic": traffic,
            "per_launch": {"marks": marks_per_launch, "avg_ms": per_launch_ms,
                           "launches_per_step": kt["launches_per_step"]}}
    rates = None if args.no_unit_rates else unit_rates()
    if rates is not None and main_rec["l"] == 20:
        # the LDS atomics actually issued (wheel and masks leave out about half the
        # algorithmic marks) against the measured random-address ds_or_b32 rate
        ex = marks_executed(primes, u, v) / kt["launches_per_step"]
        roof["vs_measured_lds"] = {"executed_marks": ex, "executed_per_s": ex / (per_launch_ms * 1e-3),
                                   "lds_or_random_per_s": rates["lds_or_random_per_s"],
                                   "frac": ex / (per_launch_ms * 1e-3) / rates["lds_or_random_per_s"]}
    also = {}
    for name in [x for x in args.also.split(",") if x and x != "none"]:
        rec = run_plain(name, max(3, args.steps // 4), 2)
        pr = rec.pop("_primes")
        rec["large_prime_hits"] = large_hits(pr, rec["u"], rec["v"], 1 << 20)
        also[name] = rec
    out = {
        "metric": "sieved numbers/sec at 1 GPU (batched vs plain, bit-exact); p99 latency",
        "value": main_rec["numbers_per_s"], "unit": "numbers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "%s: l=%d f=%d n=%d B=%d (u=%d, v=%d; 2^33 numbers centred at 1e12, plain sieve)"
                   % (args.workload, main_rec["l"], main_rec["f"], main_rec["n"], main_rec["B"], u, v),
                   "mode": "plain (one sieve_init per step, prime generation included)"},
        "p50_ms": main_rec["p50_ms"], "p99_ms": main_rec["p99_ms"],
        "ms_per_step_with_kernel_events": main_rec["ms_per_step_with_kernel_events"],
        "bit_exact": main_rec.get("bit_exact"),
        "roofline": roof,
        "kernels_ms_per_step": {k: round(x["total_ms"], 4) for k, x in main_rec["kernels"].items()},
        "also": {k: {kk: vv for kk, vv in r.items() if kk in ("numbers_per_s", "ms_per_step", "p50_ms", "p99_ms",
                                                               "bit_exact", "B", "large_prime_hits")}
                 | {"kernels_ms_per_step": {kk: round(x["total_ms"], 4) for kk, x in r["kernels"].items()}}
                 for k, r in also.items()},
    }
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    tune = None
    if args.batch_steps > 0:
        out["batch"] = run_batch_bench(args.batch_steps, log)
        tune = out["batch"]["tune"]
    if args.serve_seconds > 0:
        out["serving"] = run_serving_bench(args.serve_seconds, tune)
    if rates is not None:
        out["unit_rates"] = rates
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(main_rec["l"], main_rec["f"], main_rec["n"], main_rec["B"])
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(main_rec["l"], main_rec["f"], main_rec["n"],
                                                               main_rec["B"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
