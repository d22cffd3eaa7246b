"""Compile the C oracle (test infrastructure only).

gcc -O2 without -ffast-math: the acceptance thresholds must come from libm
exp in IEEE double precision.  OpenMP parallelises over the rows of one
sublattice, which does not change any result.
"""

from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "isf_oracle.c")
_LIB = os.path.join(_HERE, "libisf_oracle.so")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


if __name__ == "__main__":
    print(build_oracle())
