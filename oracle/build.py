"""Compile the FP64 oracle (test infrastructure) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    src = os.path.join(HERE, "oracle.c")
    if (not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(src)
            and os.path.exists(LIB_OMP)):
        return LIB
    tmp = LIB + ".tmp"
    # plain -O2: no fast-math, no FMA contraction on the default x86-64 target
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB)
    # the multi-core driver (its own library; it compiles oracle.c itself)
    tmp = LIB_OMP + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-fopenmp",
                           "-o", tmp, os.path.join(HERE, "oracle_omp.c"), "-lm"])
    os.replace(tmp, LIB_OMP)
    return LIB


if __name__ == "__main__":
    print(build())
