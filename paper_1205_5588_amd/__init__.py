"""MI355X-native Metropolis Monte Carlo of the Ising model on FCC films built
from surface height maps (Kapitan & Nefedev): hysteresis ramps and
temperature scans, plain, batched and served.

The compute path is the HIP library libisf.so (C ABI in include/isf.h);
this package is a thin binding plus the serving loop and the autotuner.
Importing the package does not load the library; the first call does.
"""

from ._lib import (BATCH_PERSISTENT, BATCH_PHASE_LAUNCH, FORMAT_BITPACK, FORMAT_INT8, INIT_DOWN, INIT_RANDOM,
                   INIT_UP, MAX_STEPS, IsfError)

__all__ = ["BATCH_PERSISTENT", "BATCH_PHASE_LAUNCH", "FORMAT_BITPACK", "FORMAT_INT8", "INIT_DOWN", "INIT_RANDOM",
           "INIT_UP", "MAX_STEPS", "IsfError"]


def __getattr__(name):
    if name in ("Lattice", "Batch", "threshold_table", "lattice_bytes"):
        from . import lattice

        return getattr(lattice, name)
    raise AttributeError(name)
