"""Compile the oracle's C source into ``oracle/_motif_oracle.so`` (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "motif_oracle.c")
LIB = os.path.join(HERE, "_motif_oracle.so")
SRC5 = os.path.join(HERE, "motif5_oracle.c")
LIB5 = os.path.join(HERE, "_motif5_oracle.so")


def _compile(src, lib, verbose):
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-Wall", "-Wextra", "-fPIC", "-shared", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _compile(SRC5, LIB5, verbose)
    return _compile(SRC, LIB, verbose)


def ensure_built(lib: str = LIB) -> str:
    src = SRC5 if lib == LIB5 else SRC
    if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        _compile(src, lib, False)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
