"""The allocation-free entry point (include/sieve.h: sieve_init_noalloc) against
sieve_init: identical tables and counts, bit for bit, on calls in a row whose
sizes shrink (the static scratch keeps the previous call's contents), and no
device memory taken by the calls themselves."""
import math

import numpy as np
import pytest

from tests.gpu_util import say, first_diff

pytestmark = pytest.mark.gpu


def _run(fn, l, f, n, B):
    import torch
    from paper_1111_3297_amd import api
    S, c = api.alloc(l, n)
    S.fill_(-1)
    c.fill_(-1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    fn(l, f, n, B, S, c)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return S.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32), free0 - free1


def test_noalloc_matches_sieve_init_on_shrinking_calls():
    from paper_1111_3297_amd import api, workloads
    l, f, n, B = workloads.plain_configs()["interval_1e12"]
    cases = [(l, f, n, B),                     # 2^33 numbers at 1e12, B = isqrt(v): two windows
             (15, 0, 64, 2048),                # 1 .. 2^22, a smaller table after a larger one
             (20, (10**15) >> 21, 3, 10**6),   # a ragged request far up, fewer windows again
             (16, 0, 5, 65535)]                # from 1, B just below l = 16's medium bound 2^16
    for k, (l, f, n, B) in enumerate(cases):
        say("noalloc case", k, l, f, n, B)
        S0, c0, _ = _run(api.sieve_init, l, f, n, B)
        S1, c1, taken = _run(api.sieve_init_noalloc, l, f, n, B)
        assert first_diff(S1, S0) is None, (k, first_diff(S1, S0))
        assert np.array_equal(c1, c0), k
        if k > 0:   # after the first call's set-up nothing is allocated
            assert taken == 0, (k, taken)


def test_noalloc_rejects_requests_beyond_its_scratch():
    from paper_1111_3297_amd import _lib
    lib = _lib.load()
    for (l, f, n, B) in [(20, (10**12) >> 21, 4, 1 << 20),        # B at the medium bound: buckets needed
                         (15, 0, 4, 1 << 15),                       # l = 15: medium bound 2^15
                         (20, 0, 8192 + 1, 1000)]:                  # more than four 2^31-bit windows
        assert lib.sieve_init_noalloc(l, f, n, B, 16, 16, None) == -8, (l, f, n, B)
