#!/usr/bin/env python3
"""Throughput of the fluctuating non-ideal D3Q19 lattice-Boltzmann step on one GPU.

Headline: million lattice-site updates per second (MLUPS) of the plain
256^3 lattice (FP32 storage), every step being the whole hot path: pull,
density halo, chemical potential, force, Philox noise, moment-space
collision, store, and every 10th step the FP64 block moments and axis
structure factor.  Inputs are synthetic (seeded initial density), resident in
device memory before the timed region.

Also reported on the same line:
  roofline      the fused step kernel against the 8 TB/s HBM peak, with
                152 algorithmic bytes per site update (19 FP32 populations
                read + 19 written), timed with HIP events on its stream, and
                against a 1 GiB device-to-device copy timed on the same GPU;
                beside it the HBM traffic and VALU busy fraction from the
                committed counter summaries (null when those were taken on
                other code or another plan);
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload;
  batched       the 96-replica finite-size sweep in one handle against the
                same 96 replicas run one after another (same seeds and steps,
                so the results are identical).

  paper_model   short runs of the paper's own model (the GL pressure in the
                equilibrium) on D3Q19 256^3 and D2Q9 256^2 and 2048^2, each
                on its default plan with its roofline.
  precision_variant
                the 512^3 lattice with FP16 deviation storage beside FP32
                storage, each on its default plan: whole steps with a
                sample every 10, and the step kernel's roofline (76 and 152
                algorithmic bytes per site update).

--workload d3q19_256_eq | d2q9_256 | d2q9_2048 times one of those alone, with
its own JSON line: the tuned plan (D3Q19), the roofline over its step
kernels and the NumPy oracle of that model on one host thread.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "split", 1: "fused", 2: "staged", 3: "rows"}
BYTES_PER_SITE = {"fp32": 152, "fp16": 76}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STEP_KERNEL_SOURCES = ("lbfss_device.hpp", "lbfss_step.hpp", "lbfss_fused.hpp")


def code_of(text):
    """C++ source without comments and whitespace: what the kernels are built
    from, so that a comment edit does not invalidate counter summaries."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "".join(text.split())


def kernel_source_hash(csrc=None, names=STEP_KERNEL_SOURCES):
    """Hash of the code the step kernels are built from (the traffic
    counters are only valid for the kernel they were taken on)."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_1202_4748_amd", "csrc")
    for name in names:
        with open(os.path.join(csrc, name)) as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(kname, workload, storage, plan):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, or None if absent, taken on other kernel sources or on
    another kernel or tile (plan: the plan dict being timed)."""
    name = workload if workload.endswith("_" + storage) else f"{workload}_{storage}"
    path = os.path.join(ROOT, "profiles", f"traffic_{kname}_{name}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    t = re.search(r"plan (\w+):(\d+):(\d+):(\d+):\d+", text)
    if not m or not b or not t or m.group(1) != kernel_source_hash():
        return None
    here = (KERNEL_NAMES[plan["kernel"]], plan["tile_x"], plan["tile_y"], plan["tile_z"])
    if (t.group(1), int(t.group(2)), int(t.group(3)), int(t.group(4))) != here:
        return None
    return float(b.group(1))


def read_valu_busy(kname, workload, names, plan=None):
    """VALU busy fraction of a step kernel from its committed counter summary
    (profiles/valu_<kernel>_<workload>.md), or None if absent, taken on
    other kernel sources or on another kernel or tile."""
    path = os.path.join(ROOT, "profiles", f"valu_{kname}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    v = re.search(r"valu_busy:\s*([0-9.]+)", text)
    if not m or not v or m.group(1) != kernel_source_hash(names=names):
        return None
    if plan is not None:
        t = re.search(r"plan (\w+:\d+:\d+:\d+)", text)
        if not t or t.group(1) != plan_text(plan):
            return None
    return float(v.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="d3q19_256")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16"])
    ap.add_argument("--sample-every", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only run warmup + timed steps (for profiler runs)")
    ap.add_argument("--plan", default=None,
                    help="fixed launch plan kernel:tx:ty:tz:graph_steps (kernel split|fused|staged|rows)")
    ap.add_argument("--no-paper-model", action="store_true",
                    help="leave out the short runs of the paper's own model (D3Q19 and D2Q9)")
    ap.add_argument("--no-precision-variant", action="store_true",
                    help="leave out the 512^3 FP16-against-FP32 storage runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (replica sharding, z-slab "
              "halo exchange) is a design, not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1202_4748_amd as lbf
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    wl = dict(workloads.WORKLOADS[args.workload])
    if "model" in wl:
        print(json.dumps(bench_paper_model(args, wl, torch, lbf, workloads, stream)), flush=True)
        return
    L = wl.pop("L")
    wl.pop("steps")
    wl.pop("storage", None)
    N = L ** 3
    log(f"[bench] {args.workload}: {L}^3, storage {args.storage}, sample every {args.sample_every}")
    if args.calibrate_copy:
        x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    sim = lbf.Sim(L, workloads.SEED, storage=args.storage, sample_every=args.sample_every, **wl)
    if args.plan:
        k, tx, ty, tz, g = args.plan.split(":")
        sim.set_plan(k, (int(tx), int(ty), int(tz)), int(g))
        log(f"[bench] plan {sim.plan()}")
    elif not args.no_tune and not args.kernel_only:
        sim.tune(steps=10)
        log(f"[bench] tuned plan {sim.plan()}")
    plan = sim.plan()
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = N * args.steps / dt / 1e6
    log(f"[bench] {args.steps} steps in {dt:.3f} s: {mlups:.0f} MLUPS")
    if args.kernel_only:
        print(json.dumps({"metric": "MLUPS", "value": mlups, "steps": args.steps}))
        return
    mom = sim.moments()

    # dominant kernel alone: same plan without sample steps, HIP events on its stream
    kplan = dict(plan)
    ksim = lbf.Sim(L, workloads.SEED, storage=args.storage, **wl)
    ksim.set_plan(KERNEL_NAMES[kplan["kernel"]], (kplan["tile_x"], kplan["tile_y"], kplan["tile_z"]),
                  max(kplan["graph_steps"], 20))
    ksim.step(40)
    ksim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nk = max(ksim.plan()["graph_steps"], 20) * 10
    e0.record(stream)
    ksim.step(nk)
    e1.record(stream)
    e1.synchronize()
    ms_per_launch = e0.elapsed_time(e1) / nk
    algo_bytes = BYTES_PER_SITE[args.storage] * N
    achieved = algo_bytes / (ms_per_launch * 1e-3) / 1e9
    kname = {0: "k_collide", 1: "k_fused", 2: "k_fused_staged", 3: "k_fused_staged"}[kplan["kernel"]]
    log(f"[bench] {kname}: {ms_per_launch * 1e3:.1f} us per step, {achieved:.0f} GB/s algorithmic")
    traffic = read_traffic(kname, args.workload, args.storage, kplan)
    del ksim
    copy_gbs = device_copy_gbs(torch, stream)
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s (read + write of 1 GiB)")

    result = {
        "metric": "MLUPS D3Q19 fluctuating step, % HBM roofline; batched vs plain at equal accuracy",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain D3Q19 {L}^3 ({args.workload})", "L": L, "sites": N,
                   "storage": args.storage, "sample_every": args.sample_every,
                   "params": {k: wl[k] for k in ("a", "b", "kappa", "rho_c", "kT", "tau")},
                   "plan": plan},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_site": BYTES_PER_SITE[args.storage],
                     "valu_busy": read_valu_busy(kname, args.workload if args.workload.endswith("_" + args.storage)
                                                 else f"{args.workload}_{args.storage}", STEP_KERNEL_SOURCES, kplan),
                     "us_per_launch": round(ms_per_launch * 1e3, 2),
                     "device_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "mass": mom["mass"],
    }

    if not args.no_batched:
        result["batched"] = batched_vs_plain(lbf, workloads, torch)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(L, wl)

    if not args.no_paper_model or not args.no_precision_variant:
        del sim
    if not args.no_paper_model:
        result["paper_model"] = paper_model_summary(args, torch, lbf, workloads, stream)
    if not args.no_precision_variant:
        result["precision_variant"] = precision_variant_summary(torch, lbf, workloads, stream)

    print(json.dumps(result), flush=True)


PAPER_MODEL = {
    # model: (lattice name, dimensions, populations)
    "eq": ("D3Q19", 3, 19),
    "d2q9": ("D2Q9", 2, 9),
}
PAPER_MODEL_SOURCES = {"eq": ("lbfss_device.hpp", "lbfss_step.hpp", "lbfss_fused.hpp", "lbfss_meq.hpp"),
                       "d2q9": ("lbfss_device.hpp", "lbfss_fused.hpp", "lbfss_d2q9.hpp")}


def paper_model_kernels(model, plan):
    """The kernels of one step of the paper's model under a plan."""
    if model == "d2q9":
        return ("k2_step_tiled",)
    if plan["kernel"] == 3:
        return ("k_meq_staged",)
    return ("k_density", "k_meq_collide")


def plan_text(plan):
    return f"{KERNEL_NAMES[plan['kernel']]}:{plan['tile_x']}:{plan['tile_y']}:{plan['tile_z']}"


def read_step_traffic(model, workload, kernels, plan=None):
    """HBM bytes per step of a paper-model workload from its committed
    counter summary, or None if absent, taken on other code or (D3Q19) on
    another kernel or tile."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernels[-1]}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    b = re.search(r"traffic_bytes_per_step:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_hash(names=PAPER_MODEL_SOURCES[model]):
        return None
    if plan is not None:
        t = re.search(r"plan (\w+:\d+:\d+:\d+)", text)
        if not t or t.group(1) != plan_text(plan):
            return None
    return float(b.group(1))


def bench_paper_model(args, wl, torch, lbf, workloads, stream):
    """The paper's own model (GL pressure in the equilibrium, noise with the
    local sound speed): on D3Q19 (LB_EQ_PRESSURE; the rows kernel
    k_meq_staged or the density and collide passes) or on D2Q9 (the lb2_*
    calls: one tiled kernel per step).  The roofline is taken over the
    step's kernels with the step's algorithmic bytes (populations read once
    and written once: 152 B per D3Q19 site, 72 B per D2Q9 site)."""
    model = wl.pop("model")
    lattice, dim, q = PAPER_MODEL[model]
    L = wl.pop("L")
    wl.pop("steps")
    every = wl.pop("sample_every", args.sample_every)
    N = L ** dim
    log(f"[bench] {args.workload}: the paper's model on {lattice}, L = {L}, sample every {every}")
    if args.calibrate_copy:
        x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    def make(sample_every, plan=None):
        if model == "d2q9":
            return lbf.Sim2D(L, workloads.SEED, sample_every=sample_every, **wl)
        sim = lbf.Sim(L, workloads.SEED, storage=args.storage, sample_every=sample_every, eq_pressure=True, **wl)
        if plan is not None:
            sim.set_plan(KERNEL_NAMES[plan["kernel"]], (plan["tile_x"], plan["tile_y"], plan["tile_z"]),
                         plan["graph_steps"])
        return sim

    sim = make(every)
    plan = None
    if model == "eq":
        if args.plan:
            k, tx, ty, tz, g = args.plan.split(":")
            sim.set_plan(k, (int(tx), int(ty), int(tz)), int(g))
        elif not args.no_tune and not args.kernel_only:
            sim.tune(steps=10)
        plan = sim.plan()
        log(f"[bench] plan {plan}")
    kernels = paper_model_kernels(model, plan)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mlups = N * args.steps / dt / 1e6
    log(f"[bench] {args.steps} steps in {dt:.3f} s: {mlups:.0f} MLUPS")
    if args.kernel_only:
        return {"metric": "MLUPS", "value": mlups, "steps": args.steps}
    del sim

    # the step's kernels without sampling, HIP events on their stream
    ksim = make(0, None if plan is None else dict(plan, graph_steps=max(plan["graph_steps"], 20)))
    ksim.step(40)
    ksim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nk = 400
    e0.record(stream)
    ksim.step(nk)
    e1.record(stream)
    e1.synchronize()
    ksim.sync()
    del ksim
    ms_per_step = e0.elapsed_time(e1) / nk
    bps = 2 * q * 4
    achieved = bps * N / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] {' + '.join(kernels)}: {ms_per_step * 1e3:.1f} us per step, {achieved:.0f} GB/s algorithmic")
    copy_gbs = device_copy_gbs(torch, stream)
    name = f"the paper's model on {lattice} {L}^{dim} ({args.workload})"
    result = {
        "metric": f"MLUPS {lattice} fluctuating step of the paper's model (GL pressure in the equilibrium)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "L": L, "sites": N, "storage": "fp32", "sample_every": every,
                   "params": {k: wl[k] for k in ("a", "b", "kappa", "rho_c", "kT", "tau")},
                   "plan": plan if plan is not None else "one tiled pass (64 x 4 sites per workgroup)"},
        "roofline": {"bound": "hbm", "kernel": " + ".join(kernels), "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": read_step_traffic(model, args.workload, kernels, plan), "bytes_per_site": bps,
                     "valu_busy": read_valu_busy(kernels[-1], args.workload, PAPER_MODEL_SOURCES[model], plan)
                     if len(kernels) == 1 else None,
                     "us_per_step": round(ms_per_step * 1e3, 2), "device_copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
    }
    if model == "d2q9" and L <= 512 and not args.no_batched:
        result["batched"] = d2q9_batched(lbf, workloads, torch, stream, L, wl, every)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_paper_model(model, L, wl)
    return result


def d2q9_batched(lbf, workloads, torch, stream, L, wl, every, reps=64, steps=200):
    """The paper's realizations side by side: 64 replicas of the L x L D2Q9
    lattice in one handle (one launch per step over every replica) against
    one replica in its own handle, same parameters and sample spacing; the
    first replica's state equals the lone handle's bit for bit.  Beside it
    the batch's step kernel alone (no samples) against the HBM roofline."""
    import numpy as np
    prms = [dict(wl, sample_every=every) for _ in range(reps)]
    seeds = [workloads.SEED + r for r in range(reps)]
    log(f"[bench] d2q9 batch: {reps} replicas of {L}^2")

    def timed(sim, n):
        sim.step(10)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(n)
        sim.sync()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    bat = lbf.Sim2D.batch(L, seeds, prms)
    t_bat = timed(bat, steps)
    one = lbf.Sim2D(L, seeds[0], **prms[0])
    t_one = timed(one, steps)
    same = bool(np.array_equal(bat.fields(f=True, replica=0)["f"], one.fields(f=True)["f"]))
    del bat, one
    k = lbf.Sim2D.batch(L, seeds, [dict(p, sample_every=0) for p in prms])
    k.step(20)
    k.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    k.step(100)
    e1.record(stream)
    e1.synchronize()
    k.sync()
    del k
    us = e0.elapsed_time(e1) / 100 * 1e3
    sites = reps * L * L
    achieved = 72.0 * sites / (us * 1e-6) / 1e9
    out = {"replicas": reps, "L": L, "sites": sites, "steps": steps, "sample_every": every,
           "batched_mlups": round(sites * steps / t_bat / 1e6, 1),
           "one_handle_mlups": round(L * L * steps / t_one / 1e6, 1),
           "speedup": round((sites / t_bat) / (L * L / t_one), 2), "identical_results": same,
           "kernel": "k2_step_tiled", "us_per_step": round(us, 2), "achieved": round(achieved, 1),
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    log(f"[bench] d2q9 batch {out['batched_mlups']} MLUPS vs one handle {out['one_handle_mlups']} MLUPS: "
        f"x{out['speedup']}; kernel {us:.1f} us per step ({out['frac']:.3f} of 8 TB/s)")
    return out


def paper_model_summary(args, torch, lbf, workloads, stream):
    """Short runs of the paper's own model beside the headline: each
    workload on its default plan, 200 timed steps with a sample every 10,
    the roofline of its step kernels; no CPU baseline (bench.py --workload
    <name> gives the full line)."""
    out = {}
    for name in ("d3q19_256_eq", "d2q9_256", "d2q9_2048"):
        sub = argparse.Namespace(**dict(vars(args), workload=name, steps=200, warmup=20, no_tune=True,
                                        no_cpu_baseline=True, kernel_only=False, plan=None, calibrate_copy=False,
                                        storage="fp32", no_batched=name != "d2q9_256"))
        r = bench_paper_model(sub, dict(workloads.WORKLOADS[name]), torch, lbf, workloads, stream)
        rf = r["roofline"]
        out[name] = {"value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"],
                     "sample_every": r["config"]["sample_every"], "plan": r["config"]["plan"],
                     "kernel": rf["kernel"], "us_per_step": rf["us_per_step"], "achieved": rf["achieved"],
                     "frac": rf["frac"], "traffic": rf["traffic"], "valu_busy": rf["valu_busy"]}
        if "batched" in r:
            out[name]["batched"] = r["batched"]
    return out


def precision_variant_summary(torch, lbf, workloads, stream, steps=60, warmup=10, every=10):
    """512^3 with FP16 deviation storage beside FP32 storage (same seed, the
    default plan of each): whole steps with a sample every 10 timed around
    the host clock, then the step kernel alone (graph replays, no samples)
    with HIP events on its stream against the 8 TB/s HBM peak."""
    wl = dict(workloads.WORKLOADS["d3q19_512_fp16"])
    L = wl.pop("L")
    wl.pop("steps")
    wl.pop("storage")
    N = L ** 3
    out = {"workload": f"plain D3Q19 {L}^3 (d3q19_512_fp16)", "sites": N}
    for storage in ("fp16", "fp32"):
        log(f"[bench] precision variant: {L}^3 {storage}")
        sim = lbf.Sim(L, workloads.SEED, storage=storage, sample_every=every, **wl)
        plan = sim.plan()
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mass = sim.moments()["mass"]
        del sim
        ksim = lbf.Sim(L, workloads.SEED, storage=storage, **wl)
        ksim.set_plan(KERNEL_NAMES[plan["kernel"]], (plan["tile_x"], plan["tile_y"], plan["tile_z"]), 20)
        ksim.step(20)
        ksim.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nk = 100
        e0.record(stream)
        ksim.step(nk)
        e1.record(stream)
        e1.synchronize()
        ksim.sync()
        del ksim
        us = e0.elapsed_time(e1) / nk * 1e3
        achieved = BYTES_PER_SITE[storage] * N / (us * 1e-6) / 1e9
        out[storage] = {"value": round(N * steps / dt / 1e6, 1), "unit": "MLUPS", "steps": steps,
                        "ms_per_step": round(dt / steps * 1e3, 3), "sample_every": every, "plan": plan,
                        "kernel": "k_fused_staged" if plan["kernel"] == 3 else KERNEL_NAMES[plan["kernel"]],
                        "us_per_launch": round(us, 1), "bytes_per_site": BYTES_PER_SITE[storage],
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit_roofline": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "mass": mass}
        log(f"[bench] {storage}: {out[storage]['value']} MLUPS whole step, kernel {us:.0f} us, "
            f"{out[storage]['frac']:.3f} of 8 TB/s")
    return out


def cpu_baseline_paper_model(model, L, wl, min_seconds=10.0, max_steps=200):
    """The NumPy oracle of the paper's model timed on one host thread: whole
    steps of the workload's lattice for D2Q9, of a 64^3 lattice for D3Q19
    (the oracle's cost per site does not depend on the size; 256^3 would
    take about a minute per step)."""
    from threadpoolctl import threadpool_limits
    if model == "eq":
        from oracle import d3q19_meq as M
        Ls, sites = 64, 64 ** 3
    else:
        from oracle import d2q9 as M
        Ls, sites = L, L ** 2
    log(f"[bench] cpu baseline: oracle of the paper's model, lattice {Ls}, 1 thread, >= {min_seconds:.0f} s")
    with threadpool_limits(limits=1):
        orc = M.Sim(Ls, 20120221, **wl)
        steps = 0
        t0 = time.perf_counter()
        while steps < max_steps:
            orc.step(1)
            steps += 1
            if time.perf_counter() - t0 >= min_seconds:
                break
        dt = time.perf_counter() - t0
    shape = f"{Ls}^3" if model == "eq" else f"{Ls}^2"
    return {"value": round(steps * sites / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 steps of a {shape} lattice ({steps * sites} site updates, {dt:.1f} s; "
                      "NumPy, BLAS limited to one thread)"}


def device_copy_gbs(torch, stream, nbytes=1 << 30, reps=5):
    """Bandwidth of a plain device-to-device copy on this GPU (bytes read plus
    bytes written per second), the practical ceiling a streaming kernel is
    compared with beside the nominal peak."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        y.copy_(x)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def batched_vs_plain(lbf, workloads, torch, steps=200):
    """96 replicas of the finite-size sweep in one handle against the same
    replicas advanced one handle at a time; identical seeds and steps, so
    identical results (checked on two replicas)."""
    import numpy as np
    Ls, seeds, prms = workloads.sweep_replicas()
    prms = [dict(p, sample_every=10, n_levels=2) for p in prms]
    sites = sum(L ** 3 for L in Ls)
    log(f"[bench] batched sweep: {len(Ls)} replicas, {sites} sites")
    bat = lbf.Sim.batch(Ls, seeds, prms)
    bat.tune(steps=10)
    bplan = bat.plan()
    t_before = bat.info()["step"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bat.step(steps)
    bat.sync()
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    singles = []
    for L, sd, p in zip(Ls, seeds, prms):
        s = lbf.Sim(L, sd, **p)
        s.set_plan(KERNEL_NAMES[bplan["kernel"]], (bplan["tile_x"], bplan["tile_y"], bplan["tile_z"]),
                   bplan["graph_steps"])
        singles.append(s)
    for s in singles:  # same step count as the batch before its timed region
        s.step(t_before)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in singles:
        s.step(steps)
    for s in singles:
        s.sync()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    equal = True
    for r in (0, len(Ls) - 1):
        equal &= bool(np.array_equal(bat.fields(r, f=True)["f"], singles[r].fields(f=True)["f"]))
    out = {"replicas": len(Ls), "sites": sites, "steps": steps,
           "batched_mlups": round(sites * steps / t_bat / 1e6, 1),
           "sequential_mlups": round(sites * steps / t_seq / 1e6, 1),
           "speedup": round(t_seq / t_bat, 2), "identical_results": equal, "plan": bplan}
    log(f"[bench] batched {out['batched_mlups']} MLUPS vs sequential {out['sequential_mlups']} "
        f"MLUPS: x{out['speedup']}")
    return out


def cpu_baseline(L, wl, min_seconds=10.0, max_steps=20):
    """The FP64 oracle timed on the host cores on whole steps of the same
    lattice: steps are taken until at least ``min_seconds`` have passed
    (at most ``max_steps``)."""
    import oracle
    threads = oracle.default_threads()
    log(f"[bench] cpu baseline: oracle {L}^3, {threads} threads, >= {min_seconds:.0f} s of steps")
    orc = oracle.Sim(L, 20120221, nthreads=threads, **wl)
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        orc.step(1)
        steps += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"value": round(steps * L ** 3 / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{steps} FP64 steps of the {L}^3 lattice ({steps * L ** 3} site updates, {dt:.1f} s)",
           "cpu": model}
    if threads > 1:
        # the same oracle on one thread, one step
        del orc
        one = oracle.Sim(L, 20120221, nthreads=1, **wl)
        log(f"[bench] cpu baseline: oracle {L}^3, 1 thread, 1 step")
        t0 = time.perf_counter()
        one.step(1)
        dt1 = time.perf_counter() - t0
        out["one_core"] = {"value": round(L ** 3 / dt1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                           "sample": f"1 FP64 step of the {L}^3 lattice ({dt1:.1f} s)"}
    return out


if __name__ == "__main__":
    main()
