"""The seeded input recipes reproduce their published fingerprints (interval ends,
request counts), so every run sieves the same synthetic workload."""
import math

from paper_1111_3297_amd import workloads as W


def test_plain_configs():
    cfg = W.plain_configs()
    l, f, n, B = cfg["interval_1e12"]
    assert (l, f, n) == (20, 474789, 4096)
    assert W.interval(l, f, n) == (995704700929, 1004294635520)
    assert B == math.isqrt(1004294635520) == 1002145
    l, f, n, B = cfg["interval_2p60"]
    assert W.interval(l, f, n) == (2**60 - 2**32 + 1, 2**60 + 2**32) and B == 2**30
    assert W.interval(*cfg["interval_2p22"][:3]) == (1, 2**22)
    # the serving stream's request of largest bound, as a plain workload
    l, f, n, B = cfg["serve_req6388"]
    t, f21, n21, kind = W.serving_stream(99, 200.0, 60.0)[6388]
    assert (l, f, n) == (20, f21, n21) and B == math.isqrt(W.interval(l, f, n)[1]) == 2133783848


def test_batch_fingerprint():
    reqs = W.batch_requests(1234, 256)
    assert len(reqs) == 256
    f21, n21 = reqs[0]
    assert W.interval(20, f21, n21) == (617018076168193, 617018109722624)
    bmax = max(math.isqrt(W.interval(20, f, n)[1]) for f, n in reqs)
    assert bmax == 29185459
    assert all(n >= 1 for _, n in reqs)


def test_serving_fingerprint():
    s = W.serving_stream(99, 200.0, 60.0)
    assert len(s) == 12040
    assert sum(1 for *_, k in s if k == "A") == 10834
    assert all(0 < t < 60 for t, *_ in s) and all(a[0] < b[0] for a, b in zip(s, s[1:]))
    vmax = max(W.interval(20, f, n)[1] for _, f, n, _ in s)
    assert math.isqrt(vmax) == 2133783848
