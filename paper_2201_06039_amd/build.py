"""Build liblbm.so (HIP, gfx950) in-tree.

    python -m paper_2201_06039_amd.build            # compile
    python -m paper_2201_06039_amd.build --resource  # also print VGPR/LDS use

Every HIP source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_api.hip")]
DEPS = SOURCES + [os.path.join(CSRC, "lbm_kernels.hpp"), os.path.join(INCLUDE, "lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def build(resource_usage: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + (["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []) + \
        ["-o", tmp] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(p) <= t for p in DEPS)


if __name__ == "__main__":
    print(build(resource_usage="--resource" in sys.argv))
