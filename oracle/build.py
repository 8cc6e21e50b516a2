"""Build the oracle's C library (liboracle.so) with gcc.

Portable flags only (no -march=native): the library may be built on one host
and run on another.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
