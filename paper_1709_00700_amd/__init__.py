"""MI355X-native hot path of a variant-generating query compiler (arXiv 1709.00700).

The compute lives in ``libhawk.so`` (HIP kernels for gfx950 behind the C ABI
in ``include/hawk.h``); ``hawk`` is its ctypes binding and ``datagen`` the
seeded synthetic input generator.
"""
from . import datagen  # noqa: F401

__all__ = ["datagen", "hawk"]
