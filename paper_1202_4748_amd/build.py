"""Compile the HIP library ``liblbfss.so`` for gfx950 (in-tree, under _build/)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbfss.hip")
DEPS = [os.path.join(HERE, "csrc", f) for f in
        ("lbfss_device.hpp", "lbfss_step.hpp", "lbfss_sample.hpp", "lbfss_fused.hpp", "lbfss_sk3.hpp",
         "lbfss_d2q9.hpp", "lbfss_meq.hpp")] + \
       [os.path.join(ROOT, "include", "lbfss.h")]
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblbfss.so")
ARCH = os.environ.get("LBFSS_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # one rounding per source expression in every kernel: the plans stay bit-identical
    "-ffp-contract=on",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
