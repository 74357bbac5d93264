"""Build the CPU oracle shared library (test infrastructure).

gcc, plain C99, -O2 and -ffp-contract=off so that no multiply-add is fused and
every operation rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ocean_oracle.c")
SRCS = [SRC, os.path.join(HERE, "mlp_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
