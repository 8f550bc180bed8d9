"""Build the oracle's C part (test infrastructure only).

Compiles ``wos_oracle.c`` with gcc and OpenMP into ``liboracle_wos.so`` next
to this file.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wos_oracle.c")
LIB = os.path.join(HERE, "liboracle_wos.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-D_DEFAULT_SOURCE", "-fno-fast-math", "-ffp-contract=off",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
