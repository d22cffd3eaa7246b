"""CPU oracle for the FCC-film Ising Metropolis dynamics.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
anything here; only the test suite, the smoke check and the benchmark's CPU
baseline do.  The oracle shares no code with the GPU path: it has its own
Philox4x32-10, its own threshold table and its own lattice bookkeeping, all
in plain cube coordinates.

Modules:
  cpu     -- ctypes wrapper of the plain C implementation (isf_oracle.c)
  ref     -- a second, pure-Python implementation for tiny films, plus the
             exact partition-function enumeration and transition matrices
             used to pin the first one
  physics -- closed forms used as pins (Onsager/Yang, single site, Eq. 2)
"""

from .build import build_oracle, oracle_lib_path  # noqa: F401
