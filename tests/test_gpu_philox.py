"""The device generator of the noise against the oracle's, word for word, and
the step counter beyond 2^32 and across a resumed run.

The noise of Eq. (lbnoise) (Sec. III A) is drawn from Philox4x32-10 with
counter (site, t_lo, call | domain << 16, t_hi) and key (seed_lo, seed_hi).
The oracle's generator is pinned against rocRAND's engine on the host
(``test_oracle_philox.py``); here the device's words and uniforms must equal
the oracle's bit for bit, and its Box-Muller normals (hardware log2, sqrt,
sin and cos on exact FP32 uniforms) must be within the bound derived below of
the oracle's FP64 normals.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev_rel_err, rel_err, require_gpu, say

pytestmark = pytest.mark.gpu

# Box-Muller in FP32 with the hardware base-2 logarithm, square root and
# sine/cosine in revolutions, on uniforms that are exact in FP32: measured
# worst |g_gpu - g_fp64| = 4.4e-7 over 5.4e4 normals (the radius reaches 5.8,
# where one FP32 ulp is 4.8e-7); the bound keeps a margin of about 4.5.
NORMAL_ATOL = 2e-6


def _counters():
    """>= 10^4 counters: random ones, the model's collision counters (domain
    0, calls 0..3) and initial-density counters (domain 1), at the largest
    site index (2^30 - 1) and at steps beyond 2^32."""
    rng = np.random.default_rng(4748)
    ctr = [rng.integers(0, 2**32, size=(6000, 4), dtype=np.uint64)]
    key = [rng.integers(0, 2**32, size=(6000, 2), dtype=np.uint64)]
    rows, keys = [], []
    seeds = (workloads.SEED, 0, 2**64 - 1, 0x123456789ABCDEF0)
    sites = (0, 1, 4095, 16**3 - 1, 256**3 - 1, 2**30 - 1) + tuple(int(v) for v in rng.integers(0, 2**30, 40))
    steps = (0, 1, 999, 2**31, 2**32 - 2, 2**32 - 1, 2**32, 2**32 + 1, 2**40 + 17, 2**63 - 1)
    for seed in seeds:
        for site in sites:
            for step in steps:
                for call in range(4):
                    rows.append((site, step & 0xFFFFFFFF, call, step >> 32))
                    keys.append((seed & 0xFFFFFFFF, seed >> 32))
            rows.append((site, 0, 1 << 16, 0))  # initial density, domain 1
            keys.append((seed & 0xFFFFFFFF, seed >> 32))
    ctr.append(np.array(rows, dtype=np.uint64))
    key.append(np.array(keys, dtype=np.uint64))
    edge = np.array([(0, 0, 0, 0), (2**32 - 1,) * 4], dtype=np.uint64)
    ctr.append(edge)
    key.append(np.array([(0, 0), (2**32 - 1,) * 2], dtype=np.uint64))
    return np.concatenate(ctr).astype(np.uint32), np.concatenate(key).astype(np.uint32)


def test_words_and_uniforms_bit_exact():
    lbf = require_gpu()
    ctr, key = _counters()
    n = ctr.shape[0]
    assert n >= 10**4
    say(f"philox words: {n} counters")
    words, uni, nrm = lbf.philox(ctr, key)
    ref_w = np.array([oracle.philox(c, k) for c, k in zip(ctr.tolist(), key.tolist())], dtype=np.uint32)
    bad = np.nonzero(np.any(words != ref_w, axis=1))[0]
    assert bad.size == 0, f"{bad.size} counters differ, first {ctr[bad[0]]} key {key[bad[0]]}"
    ref_u = np.array([[oracle.uniform(w) for w in row] for row in ref_w.tolist()])
    assert np.array_equal(uni.astype(np.float64), ref_u), "uniforms differ"
    # Box-Muller: radius from words 0 and 2, angle from words 1 and 3
    r0 = np.sqrt(-2.0 * np.log(ref_u[:, 0]))
    r1 = np.sqrt(-2.0 * np.log(ref_u[:, 2]))
    ref_g = np.stack([r0 * np.cos(2 * np.pi * ref_u[:, 1]), r0 * np.sin(2 * np.pi * ref_u[:, 1]),
                      r1 * np.cos(2 * np.pi * ref_u[:, 3]), r1 * np.sin(2 * np.pi * ref_u[:, 3])], axis=1)
    err = float(np.max(np.abs(nrm.astype(np.float64) - ref_g)))
    say(f"  normals: max |g_gpu - g_fp64| = {err:.2e}")
    assert err <= NORMAL_ATOL


def test_normals_match_oracle_site_normals():
    """The device normals of the model's counters equal (within the bound) the
    oracle's 16 collision normals and its initial-density normal."""
    lbf = require_gpu()
    seed = workloads.SEED
    cases = [(site, step) for site in (0, 77, 2**30 - 1) for step in (0, 5, 2**32 - 2, 2**32 + 9)]
    ctr, key = [], []
    for site, step in cases:
        for call in range(4):
            ctr.append((site, step & 0xFFFFFFFF, call, step >> 32))
            key.append((seed & 0xFFFFFFFF, seed >> 32))
    _, _, nrm = lbf.philox(np.array(ctr, dtype=np.uint64).astype(np.uint32),
                           np.array(key, dtype=np.uint64).astype(np.uint32))
    got = nrm.reshape(len(cases), 16).astype(np.float64)
    ref = np.array([oracle.site_normals(seed, site, step, 0) for site, step in cases])
    assert np.max(np.abs(got - ref)) <= NORMAL_ATOL
    _, _, n1 = lbf.philox(np.array([(9, 0, 1 << 16, 0)], dtype=np.uint32),
                          np.array([(seed & 0xFFFFFFFF, seed >> 32)], dtype=np.uint32))
    assert abs(float(n1[0, 0]) - oracle.site_normals(seed, 9, 0, 1)[0]) <= NORMAL_ATOL


def test_single_counter():
    lbf = require_gpu()
    w, u, g = lbf.philox(np.zeros((1, 4), np.uint32), np.zeros((1, 2), np.uint32))
    assert w.tolist()[0] == oracle.philox([0, 0, 0, 0], [0, 0])


M0 = workloads.MODEL


@pytest.mark.parametrize("t0,kernel,graph", [(2**32 - 2, "rows", 0), (2**32 + 3, "rows", 2),
                                             (2**32 - 1, "split", 0), (2**33 + 6, "fused", 4)])
def test_steps_beyond_2_32(t0, kernel, graph):
    """A handle whose counter is set near or beyond 2^32 steps as the oracle
    started at the same count: every step within the FP32 field bound, so the
    high word of the step enters the device counter as it does the oracle's
    (odd starts exercise the buffer exchange, graphs the device counter)."""
    lbf = require_gpu()
    L = 16
    say(f"t0={t0} {kernel} graph={graph}")
    sim = lbf.Sim(L, workloads.SEED, **M0)
    sim.set_plan(kernel, (16, 16, 8), graph_steps=graph)
    sim.set_step(t0)
    assert sim.info()["step"] == t0
    orc = oracle.Sim(L, workloads.SEED, t=t0, **M0)
    ref0 = oracle.Sim(L, workloads.SEED, **M0)
    chunk = max(graph, 1)
    for k in range(4):
        sim.step(chunk)
        orc.step(chunk)
        fg = sim.fields(rho=True, j=True, f=True)
        rho_o, j_o = orc.fields()
        e = (rel_err(fg["rho"], rho_o), rel_err(fg["j"], j_o), rel_err(fg["f"], orc.f))
        d = dev_rel_err(fg["rho"], rho_o)
        say(f"  step {orc.t}: max-relative {max(e):.2e}, deviation-relative {d:.2e}")
        assert max(e) <= 1e-5, f"step {orc.t}: {e}"
        assert d <= 1e-5, f"step {orc.t}: deviation-relative {d}"
    # the noise of these steps is not that of the low steps
    ref0.step(orc.t - t0)
    assert dev_rel_err(ref0.rho(), orc.rho()) > 0.05


@pytest.mark.parametrize("storage,kernel", [("fp32", "rows"), ("fp16", "rows"), ("fp32", "split")])
def test_resume_bit_identical(storage, kernel):
    """Stop a run, export its populations, create a new handle, import them and
    set the step: the continued run equals the uninterrupted one bit for bit."""
    lbf = require_gpu()
    L = 24
    say(f"resume {storage} {kernel}")
    prm = dict(M0, storage=storage)
    tile = (32, 8, 8)
    a = lbf.Sim(L, 11, **prm)
    a.set_plan(kernel, tile, graph_steps=4)
    a.step(37)
    f37 = a.fields(f=True, rho=False, j=False)["f"]
    b = lbf.Sim(L, 11, **prm)
    b.set_plan(kernel, tile, graph_steps=4)
    b.set_populations(f37)
    b.set_step(37)
    assert np.array_equal(b.fields(f=True, rho=False, j=False)["f"], f37)
    a.step(50)
    b.step(50)
    fa = a.fields(f=True)
    fb = b.fields(f=True)
    for k in ("rho", "j", "f"):
        assert np.array_equal(fa[k], fb[k]), k
    assert a.info()["step"] == b.info()["step"] == 87


def test_resume_accumulators_add_up():
    """The accumulators are additive: the sums of a stopped run (its due sample
    taken when read) plus those of the handle that resumes it equal the sums
    of the uninterrupted run (FP64 sums, in another order of addition)."""
    lbf = require_gpu()
    L = 16
    say("resume accumulators")
    prm = dict(M0, sample_every=5, series_capacity=32, hist_bins=16, hist_range=0.02)
    a = lbf.Sim(L, 13, **prm)
    a.step(40)
    b = lbf.Sim(L, 13, **prm)
    b.step(20)
    mb = b.moments()
    hb = b.histogram()
    f20 = b.fields(f=True, rho=False, j=False)["f"]
    c = lbf.Sim(L, 13, **prm)
    c.set_populations(f20)
    c.set_step(20)
    c.step(20)
    ma, mc = a.moments(), c.moments()
    assert mb["n_samples"] == 4 and mc["n_samples"] == 4 and ma["n_samples"] == 8
    for la, lb_, lc in zip(ma["levels"], mb["levels"], mc["levels"]):
        for k in ("m2", "m3", "m4", "abs_m", "E", "E2"):
            assert abs(la[k] - (lb_[k] + lc[k])) <= 1e-13 * abs(la[k]), (la["Lb"], k)
    assert np.allclose(ma["sk"], mb["sk"] + mc["sk"], rtol=1e-13, atol=0)
    assert np.array_equal(a.histogram(), hb + c.histogram())
    assert np.array_equal(a.fields(f=True)["f"], c.fields(f=True)["f"])
