"""Three-dimensional structure factor on the GPU (Sec. IV A, Eq. (G-comput))
and the Ornstein-Zernike fit of Eq. (CMF), against the oracle's FFT of the
same states and against the linearized model's statics."""
import numpy as np
import pytest

import linear_theory as lt
import workloads
from oracle import moments
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

M0 = workloads.MODEL


@pytest.mark.parametrize("L,every,stride", [(12, 2, 2), (16, 3, 1), (10, 1, 3)])
def test_shell_sums_match_oracle_fft(L, every, stride):
    """Shell geometry exactly, shell sums of C(k) within the FP32 snapshot's
    rounding (the GPU transforms the FP32-summed density deviation; the oracle
    the FP64 fields of the same state), the OZ fit as the oracle's on the same
    shell data."""
    lbf = require_gpu()
    say(f"sk3 L={L} every={every} stride={stride}")
    prm = dict(M0, a=0.02, b=0.1)
    sim = lbf.Sim(L, 9, sample_every=every, sk3_stride=stride, **prm)
    acc = moments.Accumulator(L, sk3=True)
    period = every * stride
    for _ in range(5):
        sim.step(period)
        acc.add_sk3(sim.fields()["rho"])
    g = sim.sk3()
    ref = moments.shell_average(np.zeros((L, L, L)), L)
    n = len(g["modes"])
    assert n == len(ref["modes"])
    assert np.array_equal(g["modes"], ref["modes"])
    live = g["modes"] > 0
    assert np.allclose(g["k2"][live], ref["k2"][live], rtol=1e-12, atol=0)
    assert np.allclose(g["lap"][live], ref["lap"][live], rtol=1e-12, atol=0)
    assert g["n_samples"] == 5 == acc.n_sk3
    o = acc.sk3
    tol = 2e-5 * np.abs(o) + 1e-7 * np.mean(np.abs(o[1:]))
    assert np.all(np.abs(g["sum_C"] - o) <= tol), np.max(np.abs(g["sum_C"] - o) / (np.abs(o) + 1e-300))
    # the fit is the oracle's formula on the GPU's own shell sums
    for lattice in (False, True):
        fit = sim.oz_fit(k_max=1.5, lattice=lattice)
        use = live & (np.sqrt(g["k2"]) <= 1.5)
        ref_fit = moments.oz_fit(g["mean_C"], g["modes"], g["lap"] if lattice else g["k2"], prm["kT"], use)
        assert fit["n_used"] == int(use.sum())
        for k in ("chi", "C0", "A", "B"):
            assert abs(fit[k] - ref_fit[k]) <= 1e-10 * abs(ref_fit[k]), (k, fit[k], ref_fit[k])


def test_sk3_batched_equals_plain_and_graph():
    """Batch membership and graph replay do not change the shell sums."""
    lbf = require_gpu()
    say("sk3 batch")
    pa = dict(M0, sample_every=2, sk3_stride=2)
    bat = lbf.Sim.batch([12, 8], [3, 4], [pa, dict(pa, a=0.03)])
    bat.set_plan("fused", (16, 16, 8), 8)
    bat.step(16)
    alone = lbf.Sim(12, 3, **pa)
    alone.step(16)
    a, b = bat.sk3(0), alone.sk3(0)
    assert a["n_samples"] == b["n_samples"] == 4
    assert np.array_equal(a["sum_C"], b["sum_C"])
    alone.reset_moments()
    assert alone.sk3(0)["n_samples"] == 0 and not np.any(alone.sk3(0)["sum_C"])
    with pytest.raises(lbf.LBError) as e:
        lbf.Sim(12, 3, sample_every=2, **M0).sk3(0)
    assert e.value.code == lbf.LB_ESTATE


def test_oz_fit_gaussian_statics_64():
    """b = 0, a = 0.05 at 64^3: the OZ fit over the shells with k <= 0.5 of the
    GPU's C(k) matches the same fit of the linearized model's C(k) averaged
    over the same shells (chi within 5%, xi within 8%); at small k the model
    is OZ with chi = 1/a, xi^2 = kappa_eff / a, kappa_eff = kappa + 1/12."""
    lbf = require_gpu()
    L = 64
    prm = dict(M0, a=0.05, b=0.0)
    say("sk3 statics 64^3")
    sim = lbf.Sim(L, 31, sample_every=10, sk3_stride=10, **prm)
    sim.step(3000)
    sim.reset_moments()
    sim.step(12000)
    g = sim.sk3()
    assert g["n_samples"] == 120
    kmax = 0.5
    fit = sim.oz_fit(k_max=kmax, lattice=True)
    # linearized model averaged over the same shells
    sh, ns = moments.shells(L)
    m = moments.folded_modes(L)
    use = (g["modes"] > 0) & (np.sqrt(g["k2"]) <= kmax)
    theory = np.zeros(ns)
    cache = {}
    for s_ in np.nonzero(use)[0]:
        zz, yy, xx = np.nonzero(sh == s_)
        tot = 0.0
        for a_, b_, c_ in zip(m[xx], m[yy], m[zz]):
            key = tuple(sorted((abs(int(a_)), abs(int(b_)), abs(int(c_)))))
            if key not in cache:
                k = 2 * np.pi * np.array(key, dtype=float) / L
                cache[key] = lt.structure_factor(k, prm["tau"], a=prm["a"], kappa=prm["kappa"], kT=prm["kT"])
            tot += cache[key]
        theory[s_] = tot / len(xx)
    th_fit = moments.oz_fit(np.where(use, theory, 1.0), g["modes"], g["lap"], prm["kT"], use)
    say(f"  gpu chi {fit['chi']:.3f} xi {fit['xi']:.3f}; linear model chi {th_fit['chi']:.3f} xi {th_fit['xi']:.3f}")
    assert abs(fit["chi"] / th_fit["chi"] - 1) < 0.05
    assert abs(fit["xi"] / th_fit["xi"] - 1) < 0.08
    assert abs(th_fit["chi"] * prm["a"] - 1) < 0.02
