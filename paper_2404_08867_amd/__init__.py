"""MI355X-native rank-1 lattice multi-summation (plain and MDI-LR forms).

The compute path is the HIP library ``libqmc.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/qmc.h``; ``qmc`` is its thin ctypes binding.
The binding loads the library on first use and raises if it is missing.
"""
from . import workloads  # noqa: F401  (pure input generators, no GPU needed)

__all__ = ["workloads"]
