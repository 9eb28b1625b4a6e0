"""Build the oracle's shared library (plain C, gcc, OpenMP).

Test infrastructure: the product library never builds against or loads it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "ftlm_oracle.c"), os.path.join(HERE, "spin_oracle.c"), os.path.join(HERE, "paper_cpu.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    """Compile liboracle.so next to its source; returns the library path."""
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(f) for f in SRCS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           *SRCS, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
