"""CPU checks of the C ABI: the library loads, exports every entry point that
include/sieve.h declares, and rejects invalid arguments before touching HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sieve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sieve_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_and_binding_agree():
    from paper_1111_3297_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol():
    from paper_1111_3297_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_without_gpu():
    from paper_1111_3297_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(16)
    E = {v: k for k, v in _lib.STATUS.items()}
    assert lib.sieve_init(4, 0, 1, 3, dummy, dummy, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_init(21, 0, 1, 3, dummy, dummy, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_init(10, 0, 0, 3, dummy, dummy, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_init(10, 0, 1, 2, dummy, dummy, None) == E["SIEVE_E_BOUND"]
    assert lib.sieve_init(10, 0, 1, 1 << 32, dummy, dummy, None) == E["SIEVE_E_BOUND"]
    rate = ctypes.c_double(0)
    assert lib.sieve_microbench(4, 10, ctypes.byref(rate), None) == E["SIEVE_E_ARG"]
    assert lib.sieve_microbench(0, 0, ctypes.byref(rate), None) == E["SIEVE_E_ARG"]
    assert lib.sieve_microbench(0, (1 << 20) + 1, ctypes.byref(rate), None) == E["SIEVE_E_ARG"]
    assert lib.sieve_microbench(2, 10, None, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_init(20, 1 << 43, 1, 3, dummy, dummy, None) == E["SIEVE_E_RANGE"]
    assert lib.sieve_init(10, 0, 1, 3, None, dummy, None) == E["SIEVE_E_ARG"]
    B = ctypes.c_uint64()
    assert lib.sieve_required_bound(20, 474789, 4096, ctypes.byref(B)) == 0
    assert B.value == 1002145
    assert lib.sieve_required_bound(20, 2**39 - 2048, 4096, ctypes.byref(B)) == 0
    assert B.value == 2**30 + 1
    assert _lib.strerror(-3).startswith("sieving bound")
    # the allocation-free entry point rejects what its static scratch cannot hold
    assert lib.sieve_init_noalloc(20, 474789, 4, 1 << 20, dummy, dummy, None) == E["SIEVE_E_SCRATCH"]
    assert lib.sieve_init_noalloc(15, 0, 4, 1 << 15, dummy, dummy, None) == E["SIEVE_E_SCRATCH"]
    assert lib.sieve_init_noalloc(20, 0, 8193, 1000, dummy, dummy, None) == E["SIEVE_E_SCRATCH"]
    assert lib.sieve_init_noalloc(20, 0, 1, 1000, None, dummy, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_init_noalloc(10, 0, 1, 2, dummy, dummy, None) == E["SIEVE_E_BOUND"]
    # intervals beyond 2^64: checked before the context is used
    ctx = ctypes.c_void_p()
    assert lib.sieve_ctx_create(ctypes.byref(ctx)) == 0
    M = (1 << 64) - 1
    assert lib.sieve_wide(ctx, 12, (2**51 - 1) & M, 0, 4, 1000, dummy, dummy, None, None) == E["SIEVE_E_RANGE"]
    assert lib.sieve_wide(ctx, 12, (2**115 - 4) & M, (2**115 - 4) >> 64, 4, 1000, dummy, dummy,
                          None, None) == E["SIEVE_E_RANGE"]
    assert lib.sieve_wide(ctx, 12, 0, 1 << 52, 4, 1000, dummy, dummy, None, None) == E["SIEVE_E_RANGE"]
    assert lib.sieve_wide(ctx, 12, 2**51, 0, 4, 2**40 + 1, dummy, dummy, None, None) == E["SIEVE_E_BOUND"]
    assert lib.sieve_wide(ctx, 12, 2**51, 0, 4, 2, dummy, dummy, None, None) == E["SIEVE_E_BOUND"]
    assert lib.sieve_wide(ctx, 12, 2**51, 0, 0, 1000, dummy, dummy, None, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_wide(ctx, 21, 2**51, 0, 4, 1000, dummy, dummy, None, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_wide(ctx, 10, 2**53, 0, 2**30, 1000, dummy, dummy, None, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_wide(ctx, 12, 2**51, 0, 4, 1000, None, dummy, None, None) == E["SIEVE_E_ARG"]
    assert lib.sieve_wide(None, 12, 2**51, 0, 4, 1000, dummy, dummy, None, None) == E["SIEVE_E_ARG"]
    # the wide_* tuning fields: out of range is an argument error
    for bad in ({"wide_list": 3}, {"wide_slot_log2": 5}, {"wide_slot_log2": 14}, {"wide_sort_hits": 15},
                {"wide_sort_hits": 65537}):
        t = _lib.Tune()
        for k, v in bad.items():
            setattr(t, k, v)
        assert lib.sieve_wide(ctx, 12, 2**51, 0, 4, 2**33, dummy, dummy, ctypes.byref(t), None) == E["SIEVE_E_ARG"], bad
    assert lib.sieve_ctx_destroy(ctx) == 0


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_1111_3297_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        _lib.load()
