"""Compile the CPU oracle (test infrastructure): liboracle.so with gcc -O3,
no FMA contraction and no fast-math, and liboracle_omp.so, the same file built
with OpenMP, which only the all-core CPU baseline loads."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hb_oracle.c")
FLAGS = ["-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
OUTPUTS = ((os.path.join(HERE, "liboracle.so"), []), (os.path.join(HERE, "liboracle_omp.so"), ["-fopenmp"]))


def build(force: bool = True) -> str:
    for out, extra in OUTPUTS:
        if force or not os.path.exists(out):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc"] + FLAGS + extra + [SRC, "-o", tmp, "-lm"])
            os.replace(tmp, out)
    return OUTPUTS[0][0]


if __name__ == "__main__":
    print(build())
