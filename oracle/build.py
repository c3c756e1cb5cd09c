"""Build the FP64 oracle shared library (test infrastructure only).

The oracle is plain C99 + OpenMP, compiled without fast-math so that every
operation is an IEEE-754 double operation in source order.  build(fp32=True)
compiles the same source in single precision (liboracle32.so), a measurement
of how a plain FP32 evaluation of the scheme drifts from the FP64 oracle.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB32 = os.path.join(HERE, "liboracle32.so")


def library(fp32: bool = False) -> str:
    return LIB32 if fp32 else LIB


def build(force: bool = True, fp32: bool = False) -> str:
    """Compile lbm_oracle.c -> liboracle.so (liboracle32.so with fp32) and
    return the library path."""
    lib = library(fp32)
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    extra = ["-DORC_FP32", "-fsingle-precision-constant"] if fp32 else []
    cmd = ["gcc", "-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"] + extra + ["-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
    print(build(fp32=True))
