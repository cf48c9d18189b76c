"""MI355X (gfx950) segmented odd-only sieve of Eratosthenes.

Implements the data-parallel hot path of Jarai & Vatai, "Cache optimized linear
sieve" (2011): the sieve table of Definition 1 (Section 1.3) over the interval of
Section 1.2.1, computed by hand-written HIP kernels behind the C ABI declared in
``include/sieve.h``.  The Python layer only marshals arguments (see ``_lib``).

Submodules are imported lazily so that ``workloads`` (seeded input generators)
can be used without loading the GPU library.
"""

__all__ = ["sieve", "workloads"]


def __getattr__(name):
    if name == "sieve":
        from . import api
        return api
    raise AttributeError(name)
