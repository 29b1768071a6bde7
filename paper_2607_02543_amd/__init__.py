"""ETALE dynamic graph ANN index for AMD Instinct MI355X (gfx950).

The index itself lives in libetale.so (HIP kernels behind the C ABI of
include/etale.h); ``etale`` is its Python binding and ``datagen`` draws the
seeded synthetic workloads.
"""

from . import datagen  # noqa: F401

__all__ = ["datagen", "etale"]
