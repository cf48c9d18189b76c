"""Thin Python API over the C ABI (include/sieve.h).

PyTorch provides device memory and streams; every computation happens in the HIP
kernels of libsieve.so.  Tensors passed in are int32 CUDA tensors whose storage is
read as uint32 words.
"""
import ctypes

import torch

from . import _lib as L


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, L.Tune):
        return ctypes.pointer(tune)
    t = L.Tune()
    for k, v in dict(tune).items():
        setattr(t, k, int(v))
    return ctypes.pointer(t)


def _require_cuda_i32(t, n, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous int32 CUDA tensor" % name)
    if t.numel() < n:
        raise ValueError("%s holds %d words, needs %d" % (name, t.numel(), n))


def alloc(l, n, device="cuda"):
    """Output buffers for an (l, n) request: S (n*2^l/32 words) and counts (n)."""
    S = torch.empty((n << l) // 32, dtype=torch.int32, device=device)
    c = torch.empty(n, dtype=torch.int32, device=device)
    return S, c


def required_bound(l, f, n):
    B = ctypes.c_uint64()
    L.check(L.load().sieve_required_bound(l, f, n, ctypes.byref(B)), "sieve_required_bound")
    return B.value


def sieve_init(l, f, n, B, S, counts, stream=None):
    """One-shot sieve (include/sieve.h: sieve_init)."""
    _require_cuda_i32(S, (n << l) // 32, "S")
    _require_cuda_i32(counts, n, "counts")
    L.check(L.load().sieve_init(l, f, n, B, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                                _stream(stream)), "sieve_init")


def sieve_init_noalloc(l, f, n, B, S, counts, stream=None):
    """Allocation-free one-shot sieve (include/sieve.h: sieve_init_noalloc)."""
    _require_cuda_i32(S, (n << l) // 32, "S")
    _require_cuda_i32(counts, n, "counts")
    L.check(L.load().sieve_init_noalloc(l, f, n, B, ctypes.c_void_p(S.data_ptr()),
                                        ctypes.c_void_p(counts.data_ptr()), _stream(stream)),
            "sieve_init_noalloc")


class Context:
    """An explicit library context (include/sieve.h: sieve_ctx_*)."""

    def __init__(self, _handle=None):
        self._owned = _handle is None
        if _handle is None:
            h = ctypes.c_void_p()
            L.check(L.load().sieve_ctx_create(ctypes.byref(h)), "sieve_ctx_create")
        else:
            h = _handle
        self.h = h

    @classmethod
    def default(cls):
        """The context sieve_init uses on the current device (not destroyed by close)."""
        h = L.load().sieve_default_ctx()
        if not h:
            raise L.SieveError(-5, "sieve_default_ctx")
        return cls(_handle=ctypes.c_void_p(h))

    def close(self):
        if self.h and self._owned:
            L.load().sieve_ctx_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sieve(self, l, f, n, B, S, counts, tune=None, stream=None, primes=None):
        _require_cuda_i32(S, (n << l) // 32, "S")
        _require_cuda_i32(counts, n, "counts")
        lib = L.load()
        if primes is None:
            st = lib.sieve_ctx_sieve(self.h, l, f, n, B, ctypes.c_void_p(S.data_ptr()),
                                     ctypes.c_void_p(counts.data_ptr()), _tune(tune), _stream(stream))
        else:
            st = lib.sieve_ctx_sieve_with(self.h, primes.h, l, f, n, B, ctypes.c_void_p(S.data_ptr()),
                                          ctypes.c_void_p(counts.data_ptr()), _tune(tune), _stream(stream))
        L.check(st, "sieve_ctx_sieve")

    def batch(self, primes, l, reqs, tune=None, stream=None):
        """reqs: list of (f, n, B, S, counts) with CUDA int32 tensors."""
        arr = (L.Req * max(1, len(reqs)))()
        for i, (f, n, B, S, c) in enumerate(reqs):
            _require_cuda_i32(S, (n << l) // 32, "S")
            _require_cuda_i32(c, n, "counts")
            arr[i] = L.Req(f, n, B, S.data_ptr(), c.data_ptr())
        L.check(L.load().sieve_batch(self.h, primes.h, l, arr, len(reqs), _tune(tune), _stream(stream)),
                "sieve_batch")

    def batch_scratch_bytes(self, primes, l, reqs, tune=None):
        arr = (L.Req * max(1, len(reqs)))()
        for i, (f, n, B) in enumerate(reqs):
            arr[i] = L.Req(f, n, B, None, None)
        out = ctypes.c_uint64()
        L.check(L.load().sieve_batch_scratch_bytes(primes.h, l, arr, len(reqs), _tune(tune), ctypes.byref(out)),
                "sieve_batch_scratch_bytes")
        return out.value

    def goldbach(self, primes, l, f, n, S, Q, per_number=False, stream=None):
        """Goldbach check of the even numbers of the table S of (l, f, n) against the
        odd primes q <= Q (include/sieve.h: sieve_goldbach).  Returns CUDA tensors
        (maxq int32[n], argk int64[n], fails int32[n], minq int32[n*2^l] or None),
        enqueued on the stream."""
        _require_cuda_i32(S, (n << l) // 32, "S")
        maxq = torch.empty(n, dtype=torch.int32, device=S.device)
        argk = torch.empty(n, dtype=torch.int64, device=S.device)
        fails = torch.empty(n, dtype=torch.int32, device=S.device)
        minq = torch.empty(n << l, dtype=torch.int32, device=S.device) if per_number else None
        L.check(L.load().sieve_goldbach(self.h, primes.h, l, f, n, ctypes.c_void_p(S.data_ptr()), Q,
                                        ctypes.c_void_p(maxq.data_ptr()), ctypes.c_void_p(argk.data_ptr()),
                                        ctypes.c_void_p(fails.data_ptr()),
                                        ctypes.c_void_p(minq.data_ptr()) if per_number else None, _stream(stream)),
                "sieve_goldbach")
        return maxq, argk, fails, minq

    def logsieve(self, l, f, n, B, T, C, counts, A=None, primes=None, tune=None, stream=None):
        """Log-add sieve of the odd numbers of (l, f, n) by the odd primes p <= B
        (include/sieve.h: sieve_logsieve): C (int32 words) gets the candidates with
        sum >= T, counts their number per segment, A (uint8[n*2^l], optional) the sums."""
        _require_cuda_i32(C, (n << l) // 32, "C")
        _require_cuda_i32(counts, n, "counts")
        if A is not None and not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.uint8
                                  and A.is_contiguous() and A.numel() >= (n << l)):
            raise TypeError("A must be a contiguous uint8 CUDA tensor of n*2^l bytes")
        L.check(L.load().sieve_logsieve(self.h, primes.h if primes is not None else None, l, f, n, B, T,
                                        ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                                        ctypes.c_void_p(A.data_ptr()) if A is not None else None, _tune(tune),
                                        _stream(stream)), "sieve_logsieve")

    def wide(self, l, f, n, B, S, counts, stream=None, tune=None):
        """Definition 1 for an interval beyond 2^64 (include/sieve.h: sieve_wide): f is
        a Python int below 2^(127-l) with f*2^l >= 2^63, B <= 2^40; S and counts as
        for sieve(); tune may set the wide_* fields."""
        _require_cuda_i32(S, (n << l) // 32, "S")
        _require_cuda_i32(counts, n, "counts")
        if f < 0 or f >> 128:
            raise ValueError("f must be a non-negative integer below 2^128")
        L.check(L.load().sieve_wide(self.h, l, f & (2**64 - 1), f >> 64, n, B, ctypes.c_void_p(S.data_ptr()),
                                    ctypes.c_void_p(counts.data_ptr()), _tune(tune), _stream(stream)), "sieve_wide")

    def sieve_scratch_bytes(self, l, f, n, B, tune=None, primes=None):
        """Device bytes a fresh context holds after sieve() of this request (planning pass)."""
        out = ctypes.c_uint64()
        L.check(L.load().sieve_sieve_scratch_bytes(primes.h if primes is not None else None, l, f, n, B, _tune(tune),
                                                   ctypes.byref(out)), "sieve_sieve_scratch_bytes")
        return out.value

    def scratch_bytes(self):
        """Device bytes this context's scratch buffers hold now."""
        out = ctypes.c_uint64()
        L.check(L.load().sieve_ctx_scratch_bytes(self.h, ctypes.byref(out)), "sieve_ctx_scratch_bytes")
        return out.value

    def trim(self):
        """Free this context's scratch buffers (synchronises its last stream)."""
        L.check(L.load().sieve_ctx_trim(self.h), "sieve_ctx_trim")

    def check_device_errors(self):
        L.check(L.load().sieve_check_device_errors(self.h), "sieve_check_device_errors")

    def set_timing(self, on):
        L.check(L.load().sieve_ctx_set_timing(self.h, 1 if on else 0), "sieve_ctx_set_timing")

    def kernel_times(self):
        """{kernel name: (total ms, launches)} since the last call; synchronises."""
        cap = 64
        names = (ctypes.c_char * 48 * cap)()
        ms = (ctypes.c_double * cap)()
        nl = (ctypes.c_uint64 * cap)()
        cnt = ctypes.c_uint32()
        L.check(L.load().sieve_ctx_kernel_times(self.h, names, ms, nl, cap, ctypes.byref(cnt)),
                "sieve_ctx_kernel_times")
        out = {}
        for i in range(min(cnt.value, cap)):
            out[bytes(names[i]).split(b"\0")[0].decode()] = (ms[i], nl[i])
        return out


class Primes:
    """A device sieving-prime table (include/sieve.h: sieve_primes_*)."""

    def __init__(self, B, stream=None):
        h = ctypes.c_void_p()
        L.check(L.load().sieve_primes_create(B, _stream(stream), ctypes.byref(h)), "sieve_primes_create")
        self.h = h
        c, b = ctypes.c_uint64(), ctypes.c_uint64()
        L.check(L.load().sieve_primes_info(h, ctypes.byref(c), ctypes.byref(b)), "sieve_primes_info")
        self.count, self.bound = c.value, b.value

    def nbytes(self):
        """Device bytes of the table."""
        out = ctypes.c_uint64()
        L.check(L.load().sieve_primes_bytes(self.h, ctypes.byref(out)), "sieve_primes_bytes")
        return out.value

    def to_tensor(self, stream=None):
        t = torch.empty(self.count, dtype=torch.int32, device="cuda")
        L.check(L.load().sieve_primes_copy(self.h, ctypes.c_void_p(t.data_ptr()), self.count, _stream(stream)),
                "sieve_primes_copy")
        return t

    def close(self):
        if self.h:
            L.load().sieve_primes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_buckets(l, f, n, B, tune=None, entry_cap=1 << 26):
    """First chunk's bucket layout (include/sieve.h: sieve_debug_buckets); synchronises."""
    import numpy as np
    nbins, blog, cb, nl, ne, pad = (ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64(),
                                    ctypes.c_uint64(), ctypes.c_uint32())
    bins = np.zeros(1 << 16, dtype=np.uint32)
    ent = np.zeros(entry_cap, dtype=np.uint32)
    L.check(L.load().sieve_debug_buckets(l, f, n, B, _tune(tune), bins.ctypes.data_as(ctypes.c_void_p), bins.size,
                                         ent.ctypes.data_as(ctypes.c_void_p), entry_cap, ctypes.byref(nbins),
                                         ctypes.byref(blog), ctypes.byref(cb), ctypes.byref(nl), ctypes.byref(ne),
                                         ctypes.byref(pad)),
            "sieve_debug_buckets")
    return {"bin_start": bins[:nbins.value + 1].copy(), "entries": ent[:min(ne.value, entry_cap)].copy(),
            "bin_log2": blog.value, "chunk_bits": cb.value, "nlarge": nl.value, "nentries": ne.value,
            "pad_per_bin": pad.value}


MICROBENCH = {"lds_or_random": L.MB_LDS_OR_RANDOM, "lds_or_spread": L.MB_LDS_OR_SPREAD, "valu_int32": L.MB_VALU,
              "mod64": L.MB_MOD64}


def microbench(kind, rounds=2048, stream=None):
    """Operations per second of one unit microbenchmark (include/sieve.h: sieve_microbench);
    kind is a key of MICROBENCH.  Synchronises."""
    rate = ctypes.c_double()
    L.check(L.load().sieve_microbench(MICROBENCH[kind], rounds, ctypes.byref(rate), _stream(stream)),
            "sieve_microbench")
    return rate.value
