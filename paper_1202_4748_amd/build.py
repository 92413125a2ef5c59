"""Compile the HIP library ``liblbfss.so`` for gfx950 (in-tree, under _build/)."""
import os
import re
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


# kernels whose hand-written s_waitcnt counts every vector-memory operation a
# wave issues: scratch (register spills) would add uncounted ones
COUNTED_WAIT_KERNELS = ("k_fused_staged", "k_meq_staged")


def resource_usage(remarks: str):
    """{mangled kernel name: {field: value}} from the compiler's
    kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?):\s+(\S+) \[-Rpass-analysis", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return out


def check_counted_waits(usage):
    bad = [(k, v) for k, v in usage.items() if any(n in k for n in COUNTED_WAIT_KERNELS)
           and (v.get("ScratchSize [bytes/lane]", "0") != "0" or v.get("VGPRs Spill", "0") != "0")]
    if bad:
        raise RuntimeError("kernels with counted waits use scratch memory: " +
                           ", ".join(f"{k} ({v.get('ScratchSize [bytes/lane]')} B/lane)" for k, v in bad))
    n = sum(1 for k in usage if any(c in k for c in COUNTED_WAIT_KERNELS))
    if n == 0:
        raise RuntimeError("no resource-usage remarks for the staged kernels")
    return n


# staged instances the host launches on large lattices and the waves per
# SIMD each must keep: two 512-thread workgroups per CU on 64 x 8 tiles (the
# FP32 snapshot instance is not launched there: sample steps of those plans
# run on 64 x 4 tiles), three 256-thread ones on 64 x 4
REQUIRED_OCCUPANCY = {
    "_ZN5lbfss14k_fused_stagedIfLi64ELi8ELb1ELb0E": 4,
    "_ZN5lbfss14k_fused_stagedI6__halfLi64ELi8ELb1ELb0E": 4,
    "_ZN5lbfss14k_fused_stagedI6__halfLi64ELi8ELb1ELb1E": 4,
    "_ZN5lbfss14k_fused_stagedIfLi64ELi4ELb1ELb0E": 3,
    "_ZN5lbfss14k_fused_stagedIfLi64ELi4ELb1ELb1E": 3,
}


def check_occupancy(usage):
    """Raise if a staged instance fell below the waves per SIMD its tiles
    need (a VGPR count that crept up would halve its resident workgroups)."""
    low = []
    for prefix, need in REQUIRED_OCCUPANCY.items():
        hits = [(k, v) for k, v in usage.items() if k.startswith(prefix)]
        if not hits:
            raise RuntimeError(f"no resource-usage remark for {prefix}")
        for k, v in hits:
            occ = int(v.get("Occupancy [waves/SIMD]", "0"))
            if occ < need:
                low.append(f"{k} ({v.get('VGPRs')} VGPRs, {occ} waves/SIMD, needs {need})")
    if low:
        raise RuntimeError("staged kernels below their occupancy: " + ", ".join(low))
    return len(REQUIRED_OCCUPANCY)


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-Rpass-analysis=kernel-resource-usage", "-I",
           os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    usage = resource_usage(r.stderr)
    n = check_counted_waits(usage)
    m = check_occupancy(usage)
    if verbose:
        print(f"{n} staged kernel instances without scratch memory, {m} at their occupancy", flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
