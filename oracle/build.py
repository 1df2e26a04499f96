"""Build step for the CPU oracle (test infrastructure): gcc, no FMA contraction."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle_dgemm.c"), os.path.join(HERE, "oracle_blas3.c")]

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-Wall", "-Wextra"]


def build(out: str = LIB_PATH, extra_flags=(), sources=None) -> str:
    """Compile the oracle sources into a shared library; returns its path."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", tmp, *(sources or SOURCES), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
