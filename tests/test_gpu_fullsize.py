"""Parity at the full workload sizes, in the launch configurations bench.py
times: 256^3 FP32 with the row-staged fused kernel (64 x 4 x 86 tiles, the
default plan and the tuner's usual pick at this size, and 32 x 8 x 43, the
other near-tie) replayed from a HIP graph, 512^3 with FP16 storage, and the
96-replica finite-size sweep in one handle.  The oracle runs the whole
lattice in FP64 on the host cores."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import moments
from gpu_util import rel_err, require_gpu, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

M0 = workloads.MODEL


def test_256_fp32_bench_configuration():
    lbf = require_gpu()
    L, steps = 256, 10
    say("  oracle 256^3, 10 steps")
    orc = oracle.Sim(L, workloads.SEED, **M0)
    orc.step(steps)
    rho_o, j_o = orc.fields()
    acc = moments.Accumulator(L)
    acc.add(rho_o, step=steps, j=j_o)
    # the default and tuned plan (64 x 8 tiles in four slabs; the sample step
    # runs the snapshot kernel on 64 x 4 tiles), then two other tilings
    for tile in ((64, 8, 64), (64, 4, 86), (32, 8, 43)):
        say(f"256^3 fp32 rows {tile}, graph of 10 steps, sample every 10")
        sim = lbf.Sim(L, workloads.SEED, sample_every=10, series_capacity=4, **M0)
        if tile == (64, 8, 64):
            p = sim.plan()
            assert (p["kernel"], p["tile_x"], p["tile_y"], p["tile_z"]) == (lbf.LB_KERNEL_ROWS, 64, 8, 64)
        sim.set_plan("rows", tile, 10)
        sim.step(steps)
        got = sim.fields(f=True)
        mom = sim.moments(series=True)
        e = (rel_err(got["rho"], rho_o), rel_err(got["j"], j_o), rel_err(got["f"], orc.f))
        say(f"  rel errors rho/j/f {e}")
        assert max(e) <= 1e-5
        assert mom["n_samples"] == 1
        for lv in mom["levels"]:
            ref = acc.sums[lv["Lb"]]
            for k in ("m2", "m4", "E", "E2", "abs_m"):
                assert abs(lv[k] - ref[k]) <= 2e-5 * abs(ref[k]), (lv["Lb"], k)
        # S(k) of a mode is a squared sum over planes; its FP32-trajectory error
        # is set by the typical plane-sum size, so the bound scales with mean S
        assert np.max(np.abs(mom["sk"] - acc.sk)) <= 2e-5 * np.mean(acc.sk)
        del sim


def test_512_fp16_one_step():
    """512^3, FP16 storage: the first step against the FP64 oracle (FP16
    bounds of the parity tests), and mass conserved to FP16 rounding."""
    lbf = require_gpu()
    L = 512
    say("512^3 fp16, 1 step")
    sim = lbf.Sim(L, workloads.SEED, storage="fp16", **M0)
    m0 = sim.moments()["mass"]
    sim.step(1)
    got = sim.fields(rho=True, j=True)
    say("  oracle 512^3, 1 step")
    orc = oracle.Sim(L, workloads.SEED, **M0)
    orc.step(1)
    rho_o, j_o = orc.fields()
    del orc
    e = (rel_err(got["rho"], rho_o), rel_err(got["j"], j_o))
    say(f"  rel errors rho/j {e}")
    assert e[0] <= 3e-5 and e[1] <= 1e-3
    sim.step(19)
    m1 = sim.moments()["mass"]
    assert abs(m1 - m0) / m0 < 1e-6


def test_sweep_batch_against_oracle():
    """The 96-replica sweep in one handle (fused 16x16x16 tiles, graphs):
    four replicas of different L and a against the oracle after 20 steps."""
    lbf = require_gpu()
    Ls, seeds, prms = workloads.sweep_replicas()
    say("sweep batch 96 replicas")
    bat = lbf.Sim.batch(Ls, seeds, [dict(p, sample_every=10, n_levels=2) for p in prms])
    bat.set_plan("fused", (16, 16, 16), 10)
    bat.step(20)
    for r in (0, 21, 55, 95):
        orc = oracle.Sim(Ls[r], seeds[r], **prms[r])
        orc.step(20)
        got = bat.fields(r, f=True)
        rho_o, j_o = orc.fields()
        e = (rel_err(got["rho"], rho_o), rel_err(got["j"], j_o), rel_err(got["f"], orc.f))
        assert max(e) <= 1e-5, (r, Ls[r], e)
