"""GPU serving: requests that arrive while others run are admitted into later
groups and overlap on the device; every request's result is the same as the same
request sieved alone."""
import hashlib

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_results():
    import torch
    from paper_1111_3297_amd import api, serve
    l = 20
    reqs = serve.serving_requests(l=l, limit_s=0.4)
    say("serving", len(reqs), "requests, max B", max(r.B for r in reqs))
    pr = api.Primes(max(r.B for r in reqs))
    ex = serve.GpuExecutor(pr, l, slots=3, keep_outputs=True)
    srv = serve.Server(ex, l=l, budget_bytes=64 << 30)
    res, st = srv.run(reqs)
    say("stats", st)
    assert len(res) == len(reqs)
    assert st["peak_bytes"] <= st["budget_bytes"]
    ctx = api.Context()
    for r in reqs:
        S, c = api.alloc(l, r.n)
        ctx.sieve(l, r.f, r.n, r.B, S, c, primes=pr)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint32), res[r.rid]["counts"]), r
        assert torch.equal(S, res[r.rid]["S"]), r
    ctx.check_device_errors()


def test_plain_fcfs_server_matches_batched():
    import torch
    from paper_1111_3297_amd import api, serve
    l = 20
    reqs = serve.serving_requests(l=l, limit_s=0.15)
    pr = api.Primes(max(r.B for r in reqs))
    a, _ = serve.Server(serve.PlainExecutor(pr, l), l=l, max_group=1).run(reqs)
    b, _ = serve.Server(serve.GpuExecutor(pr, l, slots=2), l=l).run(reqs)
    for r in reqs:
        assert np.array_equal(a[r.rid]["counts"], b[r.rid]["counts"]), r
