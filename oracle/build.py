"""Build the CPU oracle shared library (test infrastructure).

gcc, plain C99, -O2 and -ffp-contract=off so that no multiply-add is fused and
every operation rounds as written. A second build of the same sources with
-O3 -march=x86-64-v3 (still -ffp-contract=off, so the same arithmetic) serves
only to time the oracle as a CPU baseline; it is loaded when the environment
sets OCN_ORACLE_BUILD=o3.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ocean_oracle.c")
SRCS = [SRC, os.path.join(HERE, "mlp_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")
LIB_O3 = os.path.join(HERE, "liboracle_o3.so")
FLAGS = {"o2": ["-O2"], "o3": ["-O3", "-march=x86-64-v3"]}


def lib_path(variant: str = "o2") -> str:
    return LIB_O3 if variant == "o3" else LIB


def build(verbose: bool = False, variant: str = "o2") -> str:
    out = lib_path(variant)
    cmd = (["gcc", "-std=c99"] + FLAGS[variant] + ["-ffp-contract=off", "-fPIC", "-shared", "-Wall",
                                                    "-o", out + ".tmp"] + SRCS + ["-lm"])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build(verbose=True, variant="o3"))
