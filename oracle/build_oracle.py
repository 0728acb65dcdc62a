"""Build oracle/libmoa_oracle.so with gcc (test infrastructure only).

Flags: -ffp-contract=off keeps every product rounded before its add (no
multiply-add contraction) and no -ffast-math keeps the k order as written.
OpenMP splits rows over host threads; vector code over the contiguous j loop
does not reassociate anything.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "moa_oracle.c")
OUT = os.path.join(HERE, "libmoa_oracle.so")
FLAGS = ["-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build() -> str:
    tmp = OUT + ".tmp"
    subprocess.run(["gcc", *FLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
