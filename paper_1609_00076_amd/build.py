"""Build step for the HIP library libmdg.so (gfx950), compiled in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libmdg.so")
SOURCES = [os.path.join(PKG, "csrc", "mdg_dgemm.hip"), os.path.join(PKG, "csrc", "mdg_split.hip"),
           os.path.join(PKG, "csrc", "mdg_blas3.hip")]
INCLUDE = os.path.join(ROOT, "include")

HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument"]


def build(out: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the HIP sources into libmdg.so; returns its path."""
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPFLAGS, "-I", INCLUDE, *extra_flags, "-o", tmp, *SOURCES]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
