"""GPU observables against the oracle's plain definitions, on the same seeded
trajectories, and the mass / momentum budgets."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import moments
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

M0 = workloads.MODEL


def _oracle_run(L, seed, steps, every, n_levels, **prm):
    orc = oracle.Sim(L, seed, **prm)
    acc = moments.Accumulator(L, n_levels)
    for t in range(steps):
        orc.step(1)
        if (t + 1) % every == 0:
            rho, j = orc.fields()
            acc.add(rho, step=t + 1, j=j)
    return orc, acc


@pytest.mark.parametrize("L,n_levels,every", [(16, 0, 1), (12, 0, 3), (24, 2, 2), (10, 1, 1)])
def test_accumulators_match_oracle(L, n_levels, every):
    lbf = require_gpu()
    say(f"moments L={L} levels={n_levels} every={every}")
    steps = 30
    sim = lbf.Sim(L, 77, sample_every=every, n_levels=n_levels, series_capacity=64, **M0)
    sim.step(steps)
    got = sim.moments(series=True)
    orc, acc = _oracle_run(L, 77, steps, every, n_levels, **M0)
    assert got["n_samples"] == acc.n_samples == steps // every
    assert [lv["Lb"] for lv in got["levels"]] == acc.levels
    for lv in got["levels"]:
        ref = acc.sums[lv["Lb"]]
        assert lv["n_boxes"] * got["n_samples"] == ref["n"]
        for k in ("m2", "m4", "abs_m", "E", "E2", "m3"):
            # FP32 trajectories: moments of phi agree to ~1e-5 relative; the odd
            # moment m^3 nearly cancels, so it is held to the scale <m^2>^(3/2)
            n = ref["n"]
            scale = n * (ref["m2"] / n) ** 1.5 if k == "m3" else abs(ref[k])
            assert abs(lv[k] - ref[k]) <= 2e-5 * scale + 1e-22, (lv["Lb"], k, lv[k], ref[k])
        # boxes tile the lattice: sum of box means of phi is 0 up to rounding
        assert abs(lv["m"]) < 1e-9
    # per-mode errors scale with the typical plane-sum size (mean S), not with S(k_m)
    assert np.max(np.abs(got["sk"] - acc.sk)) <= 2e-5 * np.mean(acc.sk)
    ser = got["series"]
    assert ser.shape[0] == acc.n_samples
    # total momentum sums N per-site values whose FP32 trajectory differs from
    # the FP64 one by ~1e-7 of max |j|; the differences add up like sqrt(N)
    jscale = np.max(np.abs(orc.fields()[1]))
    ptol = 5 * np.sqrt(L ** 3) * 1e-7 * jscale
    for i, rec in enumerate(acc.series):
        assert ser[i, 0] == rec["step"]
        assert abs(ser[i, 1] - rec["mass"]) < 1e-9 * rec["mass"]
        assert np.max(np.abs(ser[i, 2:5] - rec["momentum"])) < ptol, (i, ser[i, 2:5], rec["momentum"], ptol)
        for li, Lb in enumerate(acc.levels):
            for q, k in enumerate(moments.MOMENT_KEYS):
                v, r = ser[i, 5 + 7 * li + q], rec[Lb][k]
                scale = rec[Lb]["m2"] ** 1.5 if k == "m3" else abs(r)
                assert abs(v - r) <= 2e-5 * scale + (1e-9 if k == "m" else 1e-22), (i, Lb, k, v, r)


def test_series_ring_wraps():
    lbf = require_gpu()
    say("series ring")
    sim = lbf.Sim(8, 5, sample_every=1, series_capacity=4, **M0)
    sim.step(10)
    got = sim.moments(series=True)
    assert got["n_samples"] == 10
    assert list(got["series"][:, 0]) == [7, 8, 9, 10]
    sim.reset_moments()
    sim.step(2)
    got = sim.moments(series=True)
    assert got["n_samples"] == 2 and list(got["series"][:, 0]) == [11, 12]


def test_mass_and_momentum_budget():
    """Mass is conserved up to FP32 rounding (reported in FP64); for b = 0 the
    total momentum stays zero up to rounding (exact conservation)."""
    lbf = require_gpu()
    say("budgets L=32")
    for prm in (dict(M0, b=0.0, a=0.05), M0):
        sim = lbf.Sim(32, 9, **prm)
        m0 = sim.moments()
        sim.step(500)
        m1 = sim.moments()
        N = 32 ** 3
        drift = abs(m1["mass"] - m0["mass"]) / m0["mass"]
        say(f"  b={prm['b']}: relative mass drift {drift:.2e}, momentum {m1['momentum']}")
        assert drift < 500 * N ** 0.5 * 6e-8 / N + 1e-9
        if prm["b"] == 0.0:
            assert np.max(np.abs(m1["momentum"])) < 1e-4


@pytest.mark.parametrize("kernel,graph", [("rows", 0), ("rows", 20), ("split", 10), ("fused", 20)])
def test_sample_timing_does_not_change_results(kernel, graph):
    """A sample of the state after step t is taken by the next step kernel
    (which writes the snapshot) or, when a result is read first, by a separate
    snapshot pass: both give the same bits.  Run A steps straight through
    (direct launches or graph replays), run B reads moments after every step
    so every sample is flushed; accumulators, histograms, 3D S(k) and the
    series must agree exactly."""
    lbf = require_gpu()
    L = 16
    say(f"sample timing {kernel} graph={graph}")
    prm = dict(M0, sample_every=5, series_capacity=16, hist_bins=32, hist_range=0.05, sk3_stride=2)
    a = lbf.Sim(L, 41, **prm)
    b = lbf.Sim(L, 41, **prm)
    for s_ in (a, b):
        s_.set_plan(kernel, (16, 16, 8), graph)
    a.step(40)
    for _ in range(40):
        b.step(1)
        b.moments()
    ma, mb = a.moments(series=True), b.moments(series=True)
    assert ma["n_samples"] == mb["n_samples"] == 8
    for la, lb_ in zip(ma["levels"], mb["levels"]):
        for k in ("m", "m2", "m3", "m4", "abs_m", "E", "E2"):
            assert la[k] == lb_[k], (la["Lb"], k)
    assert np.array_equal(ma["sk"], mb["sk"])
    assert np.array_equal(ma["series"], mb["series"])
    assert np.array_equal(a.histogram(), b.histogram())
    ka, kb = a.sk3(), b.sk3()
    assert ka["n_samples"] == kb["n_samples"] == 4 and np.array_equal(ka["sum_C"], kb["sum_C"])
    assert ma["series"][:, 0].tolist() == [5.0 * (i + 1) for i in range(8)]


@pytest.mark.parametrize("L,tz", [(40, 7), (128, 32)])
def test_fp32_512_thread_tiles_sample_on_their_own_tiles(L, tz):
    """FP32 rows plans on 64 x 8 tiles (512 threads) take their samples with
    the snapshot kernel on a 64 x 4 tile table of its own (three z slabs from
    L = 128 on, the plan's slabs below; L = 40 leaves partial tiles): the
    fields, accumulators, histograms and series equal those of a 64 x 4 plan
    and of the split passes bit for bit, with direct launches and graphs."""
    lbf = require_gpu()
    say(f"fp32 64x8 sampling L={L} tz={tz}")
    prm = dict(M0, sample_every=5, series_capacity=16, hist_bins=32, hist_range=0.05)
    runs = []
    for kernel, tile, g in [("split", (0, 0, 0), 0), ("rows", (64, 4, tz), 0), ("rows", (64, 8, tz), 0),
                            ("rows", (64, 8, tz), 10)]:
        s_ = lbf.Sim(L, 43, **prm)
        s_.set_plan(kernel, tile, g)
        s_.step(30)
        runs.append((s_.fields(f=True)["f"], s_.moments(series=True), s_.histogram()))
    f0, m0, h0 = runs[0]
    assert m0["n_samples"] == 6
    for f, m, h in runs[1:]:
        assert np.array_equal(f, f0)
        assert m["n_samples"] == m0["n_samples"]
        for la, lb_ in zip(m["levels"], m0["levels"]):
            for k in ("m", "m2", "m3", "m4", "abs_m", "E", "E2"):
                assert la[k] == lb_[k], (la["Lb"], k)
        assert np.array_equal(m["sk"], m0["sk"]) and np.array_equal(m["series"], m0["series"])
        assert np.array_equal(h, h0)


def test_fp32_512_thread_tiles_sample_in_a_batch():
    """A batch of FP32 replicas of different sizes on a 64 x 8 rows plan with
    graphs: its sample steps run on the snapshot tile table sized from the
    largest lattice (here 128: three slabs of 43 planes); every replica's
    fields, accumulators and series equal those of its lone handle (which
    samples on a 64 x 4 plan) bit for bit."""
    lbf = require_gpu()
    say("fp32 64x8 sampling in a batch")
    Ls, seeds = [128, 40, 64], [51, 52, 53]
    prms = [dict(M0, sample_every=5, series_capacity=16) for _ in Ls]
    prms[1]["a"] = 0.02
    bat = lbf.Sim.batch(Ls, seeds, prms)
    bat.set_plan("rows", (64, 8, 32), 10)
    bat.step(30)
    for r, (L, sd, p) in enumerate(zip(Ls, seeds, prms)):
        one = lbf.Sim(L, sd, **p)
        one.set_plan("rows", (64, 4, 16), 0)
        one.step(30)
        assert np.array_equal(bat.fields(r, f=True)["f"], one.fields(f=True)["f"]), r
        mb, mo = bat.moments(r, series=True), one.moments(series=True)
        assert mb["n_samples"] == mo["n_samples"] == 6
        for la, lb_ in zip(mb["levels"], mo["levels"]):
            for k in ("m", "m2", "m3", "m4", "abs_m", "E", "E2"):
                assert la[k] == lb_[k], (r, la["Lb"], k)
        assert np.array_equal(mb["sk"], mo["sk"]) and np.array_equal(mb["series"], mo["series"]), r
