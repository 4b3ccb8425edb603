"""Build the multi-spin-coded CPU baseline (``msc_cpu.c``) with gcc.

Generic x86-64-v2 code; the AVX-512 Philox is compiled per function and
chosen at run time when the CPU has it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msc_cpu.c")
LIB = os.path.join(HERE, "libmsc_cpu.so")


def build(force: bool = True) -> str:
    """Compile the baseline; returns the path of the shared library."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
