"""Compile the FP64 oracle (test infrastructure) into oracle/libials_oracle.so with gcc."""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "ials_oracle.c")
    out = os.path.join(_HERE, "libials_oracle.so")
    tmp = out + ".tmp"
    # x86-64-v3 (AVX2 + FMA) so the library also runs on the host of the GPU machine.
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
