"""ctypes binding of libsieve.so (include/sieve.h): argument marshalling only.

Every function here forwards to the C ABI; no step of the sieve runs in Python.
Loading fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsieve.so")

SIEVE_OK = 0
STATUS = {0: "SIEVE_OK", -1: "SIEVE_E_ARG", -2: "SIEVE_E_RANGE", -3: "SIEVE_E_BOUND",
          -4: "SIEVE_E_NOMEM", -5: "SIEVE_E_HIP", -6: "SIEVE_E_BUDGET", -7: "SIEVE_E_DEVICE",
          -8: "SIEVE_E_SCRATCH"}

# every exported entry point of include/sieve.h
EXPORTS = [
    "sieve_init", "sieve_ctx_create", "sieve_ctx_destroy", "sieve_ctx_sieve",
    "sieve_primes_create", "sieve_primes_destroy", "sieve_primes_info", "sieve_primes_copy",
    "sieve_ctx_sieve_with", "sieve_batch", "sieve_batch_scratch_bytes", "sieve_required_bound",
    "sieve_strerror", "sieve_last_hip_error", "sieve_check_device_errors", "sieve_ctx_set_timing",
    "sieve_ctx_kernel_times", "sieve_default_ctx", "sieve_copy_calibration", "sieve_microbench",
    "sieve_debug_buckets", "sieve_init_noalloc", "sieve_sieve_scratch_bytes", "sieve_ctx_scratch_bytes",
    "sieve_ctx_trim", "sieve_primes_bytes", "sieve_goldbach", "sieve_logsieve", "sieve_wide",
]
MB_LDS_OR_RANDOM, MB_LDS_OR_SPREAD, MB_VALU, MB_MOD64 = 0, 1, 2, 3


class SieveError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        name = STATUS.get(status, str(status))
        extra = ""
        if _lib is not None and status == -5:
            extra = ", hipError %d" % _lib.sieve_last_hip_error()
        super().__init__("%s failed: %s (%s%s)" % (what, name, strerror(status) if _lib else "", extra))


class Tune(ctypes.Structure):
    _fields_ = [("tile_log2", ctypes.c_uint32), ("medium_log2", ctypes.c_uint32),
                ("wave_log2", ctypes.c_uint32), ("bins_log2", ctypes.c_uint32),
                ("groups", ctypes.c_uint32), ("bin_log2", ctypes.c_uint32), ("wheel_log2", ctypes.c_uint32),
                ("ranges", ctypes.c_uint32), ("sparse", ctypes.c_uint32), ("wide_list", ctypes.c_uint32),
                ("wide_slot_log2", ctypes.c_uint32), ("wide_sort_hits", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class Req(ctypes.Structure):
    _fields_ = [("f", ctypes.c_uint64), ("n", ctypes.c_uint64), ("B", ctypes.c_uint64),
                ("S_dev", ctypes.c_void_p), ("counts_dev", ctypes.c_void_p)]


_lib = None


def load():
    """Load libsieve.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsieve.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1111_3297_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    u32, u64, vp, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    sig = {
        "sieve_init": (i32, [u32, u64, u64, u64, vp, vp, vp]),
        "sieve_init_noalloc": (i32, [u32, u64, u64, u64, vp, vp, vp]),
        "sieve_ctx_create": (i32, [ctypes.POINTER(vp)]),
        "sieve_ctx_destroy": (i32, [vp]),
        "sieve_ctx_sieve": (i32, [vp, u32, u64, u64, u64, vp, vp, ctypes.POINTER(Tune), vp]),
        "sieve_primes_create": (i32, [u64, vp, ctypes.POINTER(vp)]),
        "sieve_primes_destroy": (i32, [vp]),
        "sieve_primes_info": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "sieve_primes_copy": (i32, [vp, vp, u64, vp]),
        "sieve_ctx_sieve_with": (i32, [vp, vp, u32, u64, u64, u64, vp, vp, ctypes.POINTER(Tune), vp]),
        "sieve_batch": (i32, [vp, vp, u32, ctypes.POINTER(Req), ctypes.c_size_t, ctypes.POINTER(Tune), vp]),
        "sieve_batch_scratch_bytes": (i32, [vp, u32, ctypes.POINTER(Req), ctypes.c_size_t,
                                            ctypes.POINTER(Tune), ctypes.POINTER(u64)]),
        "sieve_sieve_scratch_bytes": (i32, [vp, u32, u64, u64, u64, ctypes.POINTER(Tune), ctypes.POINTER(u64)]),
        "sieve_ctx_scratch_bytes": (i32, [vp, ctypes.POINTER(u64)]),
        "sieve_ctx_trim": (i32, [vp]),
        "sieve_goldbach": (i32, [vp, vp, u32, u64, u64, vp, u64, vp, vp, vp, vp, vp]),
        "sieve_logsieve": (i32, [vp, vp, u32, u64, u64, u64, u32, vp, vp, vp, ctypes.POINTER(Tune), vp]),
        "sieve_wide": (i32, [vp, u32, u64, u64, u64, u64, vp, vp, ctypes.POINTER(Tune), vp]),
        "sieve_primes_bytes": (i32, [vp, ctypes.POINTER(u64)]),
        "sieve_required_bound": (i32, [u32, u64, u64, ctypes.POINTER(u64)]),
        "sieve_strerror": (ctypes.c_char_p, [i32]),
        "sieve_last_hip_error": (i32, []),
        "sieve_check_device_errors": (i32, [vp]),
        "sieve_ctx_set_timing": (i32, [vp, i32]),
        "sieve_ctx_kernel_times": (i32, [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64), u32,
                                         ctypes.POINTER(u32)]),
        "sieve_default_ctx": (vp, []),
        "sieve_copy_calibration": (i32, [vp, vp, u64, vp]),
        "sieve_microbench": (i32, [u32, u32, ctypes.POINTER(ctypes.c_double), vp]),
        "sieve_debug_buckets": (i32, [u32, u64, u64, u64, ctypes.POINTER(Tune), vp, u32, vp, u64,
                                      ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u64),
                                      ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(status):
    return load().sieve_strerror(status).decode()


def check(status, what):
    if status != SIEVE_OK:
        raise SieveError(status, what)
