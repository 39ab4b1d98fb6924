"""MI355X-native IRBSOG (random batch sum-of-Gaussians + random batch list)
force evaluation for Born-Mayer-Huggins melts (arXiv:2512.24970).

The compute path is the HIP library ``librbsog.so`` behind the C ABI declared
in ``include/rbsog.h``; :mod:`paper_2512_24970_amd.rbsog` is its ctypes
binding.  Importing this package loads nothing; the binding loads the library
on first use and raises if it is missing.
"""
__all__ = ["rbsog", "workloads", "green_kubo"]
