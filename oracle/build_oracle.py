"""Build the FP64 CPU oracle (test infrastructure only).

Two shared objects come out of the one source file:
  liboracle.so        -- `real` is double, OpenMP batch drivers enabled
  liboracle_count.so  -- `real` counts every + - * / it performs (op-count pin)
Both use -O2 -ffp-contract=off and no fast-math, so every operation is a
single correctly rounded IEEE binary64 operation in the bracketed order.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "band_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_COUNT = os.path.join(HERE, "liboracle_count.so")

_FLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> None:
    jobs = [(LIB, ["-fopenmp"]), (LIB_COUNT, ["-DORC_COUNT_FLOPS"])]
    for out, extra in jobs:
        if not force and os.path.exists(out) and \
                os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["g++", *_FLAGS, *extra, SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(force=True)
    print("built", LIB, LIB_COUNT)
