"""Order-parameter histograms P_L(m) on the GPU (Sec. II C, Eq. (PL-def)) and
the susceptibility estimates drawn from them (Eqs. (PL-highT), (PL-lowT),
(chiL), (chiL-lowT) and Gaussian fits to the peaks; Sec. IV C).

Binning turns floating point into integers, so the oracle bins the GPU's own
state (the exported fields, FP64) with its own definitions; a box whose value
lies within 1e-8 of a bin edge may legitimately land on either side (the GPU
bins the FP32-summed snapshot of the same state), and only such boxes may
move a count."""
import numpy as np
import pytest

import workloads
from oracle import moments
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

M0 = workloads.MODEL


def _oracle_hist_of_states(states, S, levels, bins, h):
    """Counts per level and, per level, how many box values sit within 1e-8
    of each bin edge (edge e between bins e - 1 and e; e = 0 and e = bins are
    the outer edges)."""
    counts = {Lb: np.zeros(bins + 2, dtype=np.int64) for Lb in levels}
    near = {Lb: np.zeros(bins + 1, dtype=np.int64) for Lb in levels}
    edges = -h + np.arange(bins + 1) * (2.0 * h / bins)
    for rho in states:
        phi = moments.order_parameter(rho)
        for Lb in levels:
            m, _ = moments.block_values(phi, S, Lb)
            counts[Lb] += moments.box_histogram(m, bins, h)
            d = np.abs(m[:, None] - edges[None, :])
            near[Lb] += np.count_nonzero(d < 1e-8, axis=0)
    return counts, near


def _assert_counts_agree(gpu, orc, near, where):
    bins = gpu.size - 2
    assert gpu.sum() == orc.sum(), where
    diff = gpu.astype(np.int64) - orc
    if not np.any(diff):
        return
    # a bin may differ by at most the edge-straddling values at its two edges
    # (under/overflow bins: the outer edges)
    allow = np.zeros(bins + 2, dtype=np.int64)
    allow[:bins] = near[:bins] + near[1:]
    allow[bins] = near[0]
    allow[bins + 1] = near[bins]
    assert np.all(np.abs(diff) <= allow), (where, np.nonzero(diff), allow[np.nonzero(diff)])


@pytest.mark.parametrize("L,bins,h", [(16, 64, 0.05), (12, 33, 0.08)])
def test_histogram_matches_oracle_binning(L, bins, h):
    lbf = require_gpu()
    every, n_samp = 3, 10
    say(f"histogram L={L} bins={bins}")
    sim = lbf.Sim(L, 21, sample_every=every, hist_bins=bins, hist_range=h, **M0)
    states = []
    for _ in range(n_samp):
        sim.step(every)
        states.append(sim.fields()["rho"])
    mom = sim.moments()
    hist = sim.histogram()
    levels = [lv["Lb"] for lv in mom["levels"]]
    assert hist.shape == (len(levels), bins + 2)
    orc, near = _oracle_hist_of_states(states, L, levels, bins, h)
    for i, Lb in enumerate(levels):
        assert hist[i].sum() == n_samp * (L // Lb) ** 3
        _assert_counts_agree(hist[i], orc[Lb], near[Lb], f"L_b={Lb}")
    # the estimates are the oracle's formulas applied to the same counts and sums
    est = sim.hist_estimates()
    kT = M0["kT"]
    for i, lv in enumerate(mom["levels"]):
        n = lv["n_boxes"] * mom["n_samples"]
        ref = moments.hist_estimates(hist[i], h, lv["Lb"], kT, n, lv["m"], lv["m2"], lv["abs_m"])
        for k, v in ref.items():
            got = est[i][k]
            # the Gaussian fit solves its least squares another way (normal
            # equations against the oracle's SVD): agreement to 1e-9
            tol = 1e-9 if k in ("m_fit", "chi_fit") else 1e-12
            if np.isinf(v) or np.isnan(v):
                assert (np.isinf(got) and np.isinf(v)) or (np.isnan(got) and np.isnan(v)), (lv["Lb"], k)
            else:
                assert abs(got - v) <= tol * max(abs(v), 1e-300), (lv["Lb"], k, got, v)


def test_histogram_batched_equals_plain_and_reset():
    """A replica's counts do not depend on its batch; reset clears them; a
    replica without histogram answers LB_ESTATE."""
    lbf = require_gpu()
    say("histogram batch")
    pa = dict(M0, sample_every=2, hist_bins=40, hist_range=0.06)
    pb = dict(M0, sample_every=2, a=0.02)
    bat = lbf.Sim.batch([20, 12], [5, 6], [pa, pb])
    bat.step(12)
    alone = lbf.Sim(20, 5, **pa)
    alone.step(12)
    assert np.array_equal(bat.histogram(0), alone.histogram(0))
    with pytest.raises(lbf.LBError) as e:
        bat.histogram(1)
    assert e.value.code == lbf.LB_ESTATE
    alone.reset_moments()
    assert not np.any(alone.histogram(0))
    with pytest.raises(lbf.LBError) as e:
        alone.hist_estimates(0)   # no sample since the reset
    assert e.value.code == lbf.LB_ESTATE
    alone.step(2)
    assert alone.histogram(0).sum(axis=1).tolist() == [(20 // lb) ** 3 for lb in (10, 5)]


def test_gaussian_histogram_estimators():
    """b = 0, a = 0.05 (Gaussian statics, far above the critical point of the
    quartic model): P_L is a Gaussian, so its centre height and a Gaussian
    fitted to it give the same chi_L as its variance (the three estimates of
    Sec. IV C: Eq. (PL-highT), the fit, Eq. (chiL)), and the variance
    matches the linearized model's box variance.  64^3, 2000 steps
    discarded, 8000 sampled every 10; L_b = 8 and 4 with 301 bins over
    +-0.04 (bin width 5-13% of the distribution's width).  Tolerance 6%: the
    centre bin holds a few 1e4 values of correlated samples."""
    import linear_theory as lt
    lbf = require_gpu()
    L = 64
    prm = dict(M0, a=0.05, b=0.0)
    say("gaussian histogram 64^3")
    sim = lbf.Sim(L, 77, sample_every=10, hist_bins=301, hist_range=0.04, **prm)
    sim.step(2000)
    sim.reset_moments()
    sim.step(8000)
    est = {e["Lb"]: e for e in sim.hist_estimates()}
    hist = sim.histogram()
    lev = [lv["Lb"] for lv in sim.moments()["levels"]]
    for Lb in (8, 4):
        e = est[Lb]
        assert hist[lev.index(Lb)][-2:].sum() == 0  # nothing outside the range
        th = lt.box_variance(L, Lb, prm["tau"], a=prm["a"], kappa=prm["kappa"], kT=prm["kT"]) * Lb ** 3 / prm["kT"]
        say(f"  L_b={Lb}: chi centre {e['chi_center']:.4g}, fit {e['chi_fit']:.4g}, variance {e['chi_var']:.4g}, "
            f"linear theory {th:.4g}, m_max {e['m_max']:.2e}")
        assert abs(e["chi_center"] / e["chi_var"] - 1) < 0.06
        assert abs(e["chi_fit"] / e["chi_var"] - 1) < 0.06
        assert abs(e["chi_var"] / th - 1) < 0.06
        assert e["m_max"] < 0.1 * np.sqrt(e["chi_var"] * prm["kT"] / Lb ** 3) + 0.04 / 301
