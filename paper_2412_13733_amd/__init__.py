"""MI355X-native hierarchical proximal Galerkin (hpG) solver.

The compute path is the HIP library ``libhpg.so`` (sources in ``csrc/``,
C ABI in ``include/hpg.h``); ``hpg`` is its thin ctypes binding.
"""
from . import hpg  # noqa: F401

__all__ = ["hpg"]
