"""MI355X-native even-odd twisted-mass clover operator and solvers.

The compute path is the HIP library ``libtmx.so`` (C-ABI, see
``include/tmx.h``); :mod:`paper_2212_06635_amd.tmx` is its thin ctypes
binding and :mod:`paper_2212_06635_amd.synth` the seeded input generator.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["synth", "tmx"]
