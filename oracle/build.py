"""Build the CPU oracle (plain C) into oracle/liboracle.so with gcc, and the
std::sort comparator into oracle/libcpusort.so with g++.

Test infrastructure: compiled by ``__graft_entry__.build()`` next to the HIP
library so the checker exists wherever the product is built.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def _compile(cmd, out, verbose):
    tmp = out + ".tmp"
    cmd = cmd + ["-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """liboracle.so (the oracle, plain C) and libcpusort.so (std::sort for the
    CPU baseline's context line)."""
    out = os.path.join(_HERE, "liboracle.so")
    _compile(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
              os.path.join(_HERE, "squaresort_oracle.c")], out, verbose)
    _compile(["g++", "-O2", "-std=c++17", "-Wall", "-fPIC", "-shared", os.path.join(_HERE, "cpu_sort.cpp")],
             os.path.join(_HERE, "libcpusort.so"), verbose)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
