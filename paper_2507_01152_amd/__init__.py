"""MI355X-native (gfx950) batched ultrasound simulator.

The compute path is the HIP library ``lib/libsonosim.so`` (C ABI in
``include/sonosim.h``); ``sonosim`` is its thin ctypes binding and
``session`` a convenience layer that keeps device copies of synthetic
workloads.  Nothing here computes the simulation on the CPU.
"""
from . import sonosim  # noqa: F401  (binding; loads the library lazily)

__all__ = ["sonosim"]
