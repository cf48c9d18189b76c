"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare it with the CPU oracle bit for bit."""
import hashlib
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_sieve(l, f, n, B, tune=None, ctx=None, primes=None):
    import torch
    from paper_1111_3297_amd import api
    S, c = api.alloc(l, n)
    if ctx is None and tune is None and primes is None:
        api.sieve_init(l, f, n, B, S, c)
        ctx = api.Context.default()
    else:
        ctx = ctx or api.Context()
        ctx.sieve(l, f, n, B, S, c, tune=tune, primes=primes)
    torch.cuda.synchronize()
    # the device error word (bucket overflow, prime-table overflow) must be clear
    ctx.check_device_errors()
    return S.cpu().numpy().view(np.uint32), c.cpu().numpy().view(np.uint32)


def sha256_words(S):
    return hashlib.sha256(np.ascontiguousarray(S).view(np.uint32).tobytes()).hexdigest()


def first_diff(a, b):
    d = np.flatnonzero(a != b)
    if d.size == 0:
        return None
    i = int(d[0])
    return "word %d: gpu %08x oracle %08x (%d words differ)" % (i, int(a[i]), int(b[i]), d.size)
