"""Build step for the FP64 CPU oracle (test infrastructure).

Compiles ``lbora.c`` into ``liblbora.so`` beside it with plain gcc: -O2, no
fast-math and no floating-point contraction, so every operation is one
IEEE-754 binary64 operation in the order the source writes it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbora.c")
LIB = os.path.join(HERE, "liblbora.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
        SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
