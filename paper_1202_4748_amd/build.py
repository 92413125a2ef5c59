"""Compile the HIP library ``liblbfss.so`` for gfx950 (in-tree, under _build/)."""
import os
import re
import subprocess
import sys
import tempfile

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


_LABEL = re.compile(r"^(\.LBB\w+):")
_LDS_DMA = re.compile(r"^(global|buffer)_load_lds")
_VMEM = re.compile(r"^(global|buffer|flat|scratch)_(load|store|atomic)")
_WAIT = re.compile(r"^s_waitcnt\b.*\bvmcnt\((\d+)\)")
_BRANCH = re.compile(r"^s_c?branch\w*\s+(\.LBB\w+)")


def asm_functions(text: str):
    """{function name: its lines} from device assembly (gfx9 syntax)."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.match(r"^([A-Za-z_][\w.$]*):", line)
        if m and not line.startswith(".L"):
            cur = out.setdefault(m.group(1), [])
            continue
        if cur is not None and line.startswith(".Lfunc_end"):
            cur = None
            continue
        if cur is not None:
            cur.append(line)
    return out


def counted_wait_shortfalls(lines):
    """Counted waits of one kernel that could return early.

    A wait s_waitcnt vmcnt(N) lets the N youngest vector-memory operations
    of the wave run on; the staged kernels use it to wait for the previous
    global->LDS copies while the collision's stores (non-temporal, `nt`)
    still run, which holds only if at least N vector-memory operations were
    issued after the last copy.  A forward pass over the control flow finds,
    for each wait with N > 0, the fewest such operations on any path from a
    copy through collision stores; paths without them are the iterations
    without a collision, which take the full wait at run time (the waits are
    chosen by whether the last iteration stored).  Stores merged, moved
    ahead of the copies or dropped leave such a path below N, or none.
    Returns [(line, N, count)] for each wait below its N (count 0: no such
    path), and the number of waits checked."""
    ins, labels = [], {}
    for raw in lines:
        t = raw.split(";")[0].strip()
        if not t:
            continue
        m = _LABEL.match(t)
        if m:
            labels[m.group(1)] = len(ins)
            ins.append(("label", m.group(1), raw))
            continue
        if t.startswith("."):
            continue
        op = t.split()[0]
        if _LDS_DMA.match(op):
            ins.append(("copy", None, raw))
        elif _VMEM.match(op):
            ins.append(("vmem", "nt" if "_store" in op and re.search(r"\bnt\b", t) else None, raw))
        elif _WAIT.match(t):
            ins.append(("wait", int(_WAIT.match(t).group(1)), raw))
        elif _BRANCH.match(t):
            ins.append(("branch", _BRANCH.match(t).group(1), raw))
        elif op in ("s_endpgm", "s_setpc_b64"):
            ins.append(("end", None, raw))
        else:
            ins.append(("other", None, raw))
    # basic blocks: they start at labels and after branches
    starts = sorted({0} | {i for i, x in enumerate(ins) if x[0] == "label"}
                    | {i + 1 for i, x in enumerate(ins) if x[0] in ("branch", "end") and i + 1 < len(ins)})
    bounds = list(zip(starts, starts[1:] + [len(ins)]))
    block_at = {b: k for k, (b, _) in enumerate(bounds)}
    succ = []
    for b, e in bounds:
        out = []
        last = ins[e - 1] if e > b else None
        if last and last[0] == "branch" and last[1] in labels:
            out.append(block_at[labels[last[1]]])
        uncond = last is not None and ((last[0] == "branch" and last[2].strip().startswith("s_branch "))
                                       or last[0] == "end")
        if not uncond and e < len(ins):
            out.append(block_at[e])
        succ.append(out)
    # state at a point: fewest operations since the last copy on a path that
    # passed collision stores (INF: none), and on a path that passed none
    INF = 1 << 30

    def run(v, b, e, report=None):
        low, zc = v
        for i in range(b, e):
            k, a, raw = ins[i]
            if k == "copy":
                low, zc = INF, 0
            elif k == "vmem":
                if a == "nt":
                    low, zc = min(low + 1, zc + 1), INF
                else:
                    low, zc = (low + 1 if low < INF else INF), (zc + 1 if zc < INF else INF)
            elif k == "wait" and a > 0 and report is not None and (low < INF or zc < INF):
                report.append((raw.strip(), a, low if low < INF else 0))
        return low, zc

    entry = [(INF, INF)] * len(bounds)
    work, seen = [0], {0}
    while work:
        k = work.pop()
        b, e = bounds[k]
        low, zc = run(entry[k], b, e)
        for t in succ[k]:
            old = entry[t]
            new = (min(old[0], low), min(old[1], zc))
            if new != old or t not in seen:
                entry[t] = new
                seen.add(t)
                work.append(t)
    waits = []
    for k, (b, e) in enumerate(bounds):
        run(entry[k], b, e, waits)
    return [w for w in waits if w[2] < w[1]], len(waits)


def check_counted_wait_order(asm: str):
    """Raise if a staged kernel's counted wait could let a copy it waits for
    still run (stores merged, moved before the copies or taken out)."""
    funcs = {k: v for k, v in asm_functions(asm).items() if any(n in k for n in COUNTED_WAIT_KERNELS)}
    if not funcs:
        raise RuntimeError("no staged kernels in the device assembly")
    problems, total = [], 0
    for name, lines in funcs.items():
        bad, checked = counted_wait_shortfalls(lines)
        total += checked
        problems += [f"{name}: {w} with {c} younger operations" for w, _, c in bad]
    if problems:
        raise RuntimeError("counted waits without enough younger operations: " + "; ".join(problems[:5]))
    return total


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
    with tempfile.TemporaryDirectory() as td:
        # the device assembly of the same source and flags, compiled alongside
        asm_path = os.path.join(td, "lbfss.s")
        acmd = [hipcc, *[f for f in HIPCC_FLAGS if f != "-shared"], *extra, "--cuda-device-only", "-S", "-I",
                os.path.join(ROOT, "include"), "-o", asm_path, SRC]
        pa = subprocess.Popen(acmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        a_out, a_err = pa.communicate()
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise subprocess.CalledProcessError(r.returncode, cmd)
        if pa.returncode != 0:
            sys.stderr.write(a_err)
            raise subprocess.CalledProcessError(pa.returncode, acmd)
        with open(asm_path) as f:
            w = check_counted_wait_order(f.read())
    usage = resource_usage(r.stderr)
    n = check_counted_waits(usage)
    m = check_occupancy(usage)
    if verbose:
        print(f"{n} staged kernel instances without scratch memory, {m} at their occupancy, "
              f"{w} counted waits behind enough younger operations", flush=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
