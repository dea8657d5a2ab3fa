"""Compile the C part of the oracle (test infrastructure) into oracle/_dirac_oracle.so.

Plain gcc with OpenMP; no architecture-specific flags, so the library built
here also runs on other x86-64 hosts.  -fcx-limited-range lets gcc inline
complex multiplication instead of calling its NaN-recovery helper.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dirac_oracle.c")
LIB = os.path.join(HERE, "_dirac_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fcx-limited-range", "-std=c11", "-fPIC", "-shared",
           SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
