"""El-WaveHoltz on MI355X: the filter-operator hot path as HIP kernels for
gfx950 behind the C ABI declared in include/elwh.h.

Importing this package is cheap; the HIP library is loaded on first use of
``paper_2205_12344_amd.elwh`` (which imports torch first, so the library
binds to the same HIP runtime as torch).
"""

__all__ = ["inputs", "elwh", "build"]
