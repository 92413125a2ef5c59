"""Compile the FP64 C oracle into ``oracle/_build/liblbfss_oracle.so`` with gcc.

Test infrastructure: the library built here is loaded only by ``tests/``, the
smoke check and the CPU-baseline leg of ``bench.py``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbfss_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblbfss_oracle.so")
# the same source with AddressSanitizer and UndefinedBehaviorSanitizer (host
# code only), loaded instead of LIB when LBFSS_ORACLE_SANITIZE=1
LIB_SAN = os.path.join(OUT_DIR, "liblbfss_oracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def library():
    return LIB_SAN if os.environ.get("LBFSS_ORACLE_SANITIZE") == "1" else LIB


def build(verbose: bool = False, sanitize: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra"] + (SAN_FLAGS if sanitize else []) + \
          ["-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
