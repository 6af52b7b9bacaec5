"""Build the CPU oracle (test infrastructure): oracle/liblbo.so from lbo.c
(D2Q9) and lbo3.c (D3Q19, D3Q27).

Plain gcc, FP64, no fast-math and no floating-point contraction, so that the
oracle's single-precision noise routines round every operation separately.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbo.so")


SOURCES = [os.path.join(HERE, "lbo.c"), os.path.join(HERE, "lbo3.c")]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-D_DEFAULT_SOURCE", *SOURCES, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
