"""Python access to the plain CPU oracle (``sieve_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use this module.  The GPU library never imports
it, and it imports nothing from the GPU package.

The oracle computes the odd-only sieve table of Definition 1 (Section 1.3) for the
interval of Section 1.2.1, u = f*2^(l+1)+1 .. v = (f+n)*2^(l+1), by marking every
odd multiple m*p (m >= 3) of every odd prime p <= B.  See the C file's header.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sieve_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force=False):
    """Compile the oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_sieve.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, u32p, u32p]
        lib.oracle_sieve.restype = ctypes.c_int
        lib.oracle_sieve_with.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          u32p, ctypes.c_long, u32p, u32p]
        lib.oracle_sieve_with.restype = ctypes.c_int
        lib.oracle_goldbach.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p, ctypes.c_uint64,
                                        u32p, u32p, ctypes.POINTER(ctypes.c_uint64), u32p]
        lib.oracle_goldbach.restype = ctypes.c_int
        lib.oracle_logsieve.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, u32p, u32p, ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_logsieve.restype = ctypes.c_int
        lib.oracle_sieve_wide.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, u32p, u32p]
        lib.oracle_sieve_wide.restype = ctypes.c_int
        lib.oracle_odd_primes64.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64))]
        lib.oracle_odd_primes64.restype = ctypes.c_longlong
        lib.oracle_odd_primes.argtypes = [ctypes.c_uint64, ctypes.POINTER(u32p)]
        lib.oracle_odd_primes.restype = ctypes.c_long
        lib.oracle_lemma1_offset.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        lib.oracle_lemma1_offset.restype = ctypes.c_uint32
        lib.oracle_lemma2_skip.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        lib.oracle_lemma2_skip.restype = ctypes.c_uint64
        lib.oracle_count_total.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint64]
        lib.oracle_count_total.restype = ctypes.c_longlong
        libc = ctypes.CDLL(None)
        libc.free.argtypes = [ctypes.c_void_p]
        lib._free = libc.free
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def sieve(l, f, n, B):
    """Definition 1: returns (S as uint32 words, counts per 2^l-bit segment)."""
    lib = _load()
    nwords = (n << l) // 32
    S = np.zeros(max(nwords, 1), dtype=np.uint32)
    c = np.zeros(max(n, 1), dtype=np.uint32)
    rc = lib.oracle_sieve(l, f, n, B,
                          S.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                          c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    if rc != 0:
        raise OracleError("oracle_sieve(l=%d, f=%d, n=%d, B=%d) -> %d" % (l, f, n, B, rc))
    return S[:nwords], c[:n]


def sieve_with(l, f, n, B, P):
    """Definition 1 with the odd primes given (ascending uint32 array holding at
    least every odd prime <= B; larger entries are ignored): (S, counts)."""
    lib = _load()
    P = np.ascontiguousarray(P, dtype=np.uint32)
    nwords = (n << l) // 32
    S = np.zeros(max(nwords, 1), dtype=np.uint32)
    c = np.zeros(max(n, 1), dtype=np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    rc = lib.oracle_sieve_with(l, f, n, B, P.ctypes.data_as(u32p), len(P),
                               S.ctypes.data_as(u32p), c.ctypes.data_as(u32p))
    if rc != 0:
        raise OracleError("oracle_sieve_with(l=%d, f=%d, n=%d, B=%d) -> %d" % (l, f, n, B, rc))
    return S[:nwords], c[:n]


def goldbach(l, f, n, S, Q, per_number=True):
    """Goldbach check of the even numbers u+1 .. v against the table S of (l, f, n)
    and the odd primes q <= Q (see oracle_goldbach in sieve_oracle.c): returns
    (minq per even number or None, maxq, argk, fails per segment)."""
    lib = _load()
    u32p = ctypes.POINTER(ctypes.c_uint32)
    S = np.ascontiguousarray(S, dtype=np.uint32)
    assert S.size >= (n << l) // 32
    minq = np.zeros(n << l, dtype=np.uint32) if per_number else None
    maxq = np.zeros(n, dtype=np.uint32)
    argk = np.zeros(n, dtype=np.uint64)
    fails = np.zeros(n, dtype=np.uint32)
    rc = lib.oracle_goldbach(l, f, n, S.ctypes.data_as(u32p), Q,
                             minq.ctypes.data_as(u32p) if per_number else None, maxq.ctypes.data_as(u32p),
                             argk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), fails.ctypes.data_as(u32p))
    if rc != 0:
        raise OracleError("oracle_goldbach(l=%d, f=%d, n=%d, Q=%d) -> %d" % (l, f, n, Q, rc))
    return minq, maxq, argk, fails


def logsieve(l, f, n, B, T, with_sums=True):
    """Log-add sieve of the odd numbers of (l, f, n) by the odd primes p <= B
    (oracle_logsieve): returns (C bit table as uint32 words, counts of ones per
    segment, the byte sums A or None)."""
    lib = _load()
    u32p = ctypes.POINTER(ctypes.c_uint32)
    nb = n << l
    C = np.zeros(max(nb // 32, 1), dtype=np.uint32)
    c = np.zeros(max(n, 1), dtype=np.uint32)
    A = np.zeros(nb, dtype=np.uint8) if with_sums else None
    rc = lib.oracle_logsieve(l, f, n, B, T, C.ctypes.data_as(u32p), c.ctypes.data_as(u32p),
                             A.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if with_sums else None)
    if rc != 0:
        raise OracleError("oracle_logsieve(l=%d, f=%d, n=%d, B=%d, T=%d) -> %d" % (l, f, n, B, T, rc))
    return C[:nb // 32], c[:n], A


def sieve_wide(l, f, n, B):
    """Definition 1 for f up to 2^127 / 2^l (intervals past 2^64) and B up to 2^40:
    returns (S as uint32 words, counts per segment)."""
    lib = _load()
    u32p = ctypes.POINTER(ctypes.c_uint32)
    nwords = (n << l) // 32
    S = np.zeros(max(nwords, 1), dtype=np.uint32)
    c = np.zeros(max(n, 1), dtype=np.uint32)
    rc = lib.oracle_sieve_wide(l, f & ((1 << 64) - 1), f >> 64, n, B, S.ctypes.data_as(u32p), c.ctypes.data_as(u32p))
    if rc != 0:
        raise OracleError("oracle_sieve_wide(l=%d, f=%d, n=%d, B=%d) -> %d" % (l, f, n, B, rc))
    return S[:nwords], c[:n]


def odd_primes64(B):
    """Odd primes 3 <= p <= B (B <= 2^40) as uint64."""
    lib = _load()
    ptr = ctypes.POINTER(ctypes.c_uint64)()
    cnt = lib.oracle_odd_primes64(B, ctypes.byref(ptr))
    if cnt < 0:
        raise OracleError("oracle_odd_primes64(%d) failed" % B)
    out = np.ctypeslib.as_array(ptr, shape=(max(cnt, 1),))[:cnt].copy()
    lib._free(ptr)
    return out


def odd_primes(B):
    """Odd primes 3 <= p <= B (plain sieve of Eratosthenes, Section 1.1)."""
    lib = _load()
    ptr = ctypes.POINTER(ctypes.c_uint32)()
    cnt = lib.oracle_odd_primes(B, ctypes.byref(ptr))
    if cnt < 0:
        raise OracleError("out of memory")
    out = np.ctypeslib.as_array(ptr, shape=(max(cnt, 1),))[:cnt].copy()
    lib._free(ptr)
    return out


def lemma1_offset(p, f, l):
    """Lemma 1 (Section 2.1): unique 0 <= q < p with p | 2(f*2^l + q) + 1."""
    return _load().oracle_lemma1_offset(p, f, l)


def lemma2_skip(p, q, l):
    """Lemma 2 (Section 2.2): number of segments skipped after a hit at offset q."""
    return _load().oracle_lemma2_skip(p, q, l)


def count_total(l, f, n, B):
    """Sum of the per-segment zero-bit counts of Definition 1's table."""
    r = _load().oracle_count_total(l, f, n, B)
    if r < 0:
        raise OracleError("oracle_count_total failed")
    return r


def interval(l, f, n):
    """Section 1.2.1: u = f*2^(l+1)+1, v = (f+n)*2^(l+1)."""
    return f * (1 << (l + 1)) + 1, (f + n) * (1 << (l + 1))
