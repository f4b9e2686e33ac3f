"""Build libenomr.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libenomr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: only the fma() calls written in the source are fused, so
# every formula rounds exactly as written.  Packed FP32 is disabled for the
# device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False):
    objs = []
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    steps = [
        ([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, "tables.cpp"), "-o", os.path.join(tmp, "tables.o")]
         + COMMON + DEVICE, os.path.join(tmp, "tables.o")),
        ([HIPCC, "-c", os.path.join(CSRC, "capi.hip"), "-o", os.path.join(tmp, "capi.o")] + COMMON + DEVICE,
         os.path.join(tmp, "capi.o")),
    ]
    for cmd, obj in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    link = [HIPCC, "-shared", "-o", LIB + ".tmp"] + objs + DEVICE + ["-fPIC"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
