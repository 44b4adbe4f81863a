"""Build the FP64 CPU oracle (test infrastructure) with gcc.

Compiled with -ffp-contract=off and without fast-math so that every
operation rounds exactly as written in double precision; -fopenmp enables
the optional multi-threaded pixel loops (one thread unless set_threads()).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "gi_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [s for s in SRC if os.path.exists(s)]
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    newest = max(os.path.getmtime(s) for s in SRC if os.path.exists(s))
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
