"""Pins of the oracle's order-parameter histogram and its susceptibility
estimates (Sec. II B-C, Eqs. (PL-def), (PL-highT), (PL-lowT), (chiL),
(chiL-lowT); Sec. IV C for the peak-height estimate) against values fixed by
hand, closed forms of Gaussian distributions and sampling."""
import math

import numpy as np
import pytest

from oracle import moments as M


def test_bin_rule_by_hand():
    # h = 1, 4 bins: edges -1, -0.5, 0, 0.5, 1; left edges belong to their bin
    vals = [-1.0, -0.5, 0.0, 0.999, 1.0, -1.0001, 0.25, -1e-300, 0.5, -0.75]
    c = M.box_histogram(vals, 4, 1.0)
    assert c.tolist() == [2, 1, 3, 2, 1, 1]   # bins 0..3, below, at-or-above
    assert c.sum() == len(vals)


def test_odd_bins_centre_bin_holds_zero():
    c = M.box_histogram([0.0, 1e-9, -1e-9], 5, 1.0)   # edges at +-0.2: all in bin 2
    assert c.tolist() == [0, 0, 3, 0, 0, 0, 0]


def _gauss_bin_probs(edges, mu, sigma):
    cdf = np.array([0.5 * (1.0 + math.erf((e - mu) / (sigma * math.sqrt(2.0)))) for e in edges])
    return np.diff(cdf)


def _counts_from_density(probs, total, under=0.0, over=0.0):
    c = np.concatenate([probs * total, [under * total, over * total]])
    return np.rint(c)


@pytest.mark.parametrize("bins,tol", [(601, 1e-4), (600, 3e-4)])
def test_centre_height_recovers_chi_of_a_gaussian(bins, tol):
    """Eq. (PL-highT): a Gaussian of variance kT chi / L^d has central height
    L^(d/2) / sqrt(2 pi kT chi); the estimate inverts that (bin averaging
    biases it by O(w^2 / sigma^2))."""
    Lb, kT, chi = 4, 1e-4, 7.5
    sigma = math.sqrt(kT * chi / Lb ** 3)
    h = 6.0 * sigma
    edges = np.linspace(-h, h, bins + 1)
    p = _gauss_bin_probs(edges, 0.0, sigma)
    tail = 0.5 * math.erfc(6.0 / math.sqrt(2.0))
    c = _counts_from_density(p, 1e13, tail, tail)
    est = M.hist_estimates(c, h, Lb, kT, n=1.0, sum_m=0.0, sum_m2=sigma ** 2, sum_abs_m=0.0)
    assert abs(est["chi_center"] / chi - 1) < tol
    assert abs(est["chi_var"] / chi - 1) < 1e-12
    assert est["m_max"] < 2.0 * h / bins


def test_peak_height_and_position_of_two_displaced_gaussians():
    """Eq. (PL-lowT): two Gaussians of variance kT chi / L^d at +-M_L, weight
    1/2 each; the peak height is L^(d/2) / (2 sqrt(2 pi kT chi)), so
    chi = L^d / (8 pi kT P_max^2), and the peak sits at M_L."""
    Lb, kT, chi, ML = 2, 1e-4, 3.0, 0.05
    sigma = math.sqrt(kT * chi / Lb ** 3)
    h, bins = 0.1, 2001
    edges = np.linspace(-h, h, bins + 1)
    p = 0.5 * (_gauss_bin_probs(edges, ML, sigma) + _gauss_bin_probs(edges, -ML, sigma))
    c = _counts_from_density(p, 1e13)
    w = 2 * h / bins
    # moments of the mixture: <m> = 0, <m^2> = ML^2 + sigma^2
    est = M.hist_estimates(c, h, Lb, kT, n=1.0, sum_m=0.0, sum_m2=ML ** 2 + sigma ** 2, sum_abs_m=ML)
    assert abs(est["m_max"] - ML) <= 0.5 * w + 1e-15
    assert abs(est["chi_peak"] / chi - 1) < 2e-3
    # Eq. (chiL-lowT) removes the displacement: <m^2> - <|m|>^2 ~ sigma^2
    assert abs(est["chi_var_low"] / chi - 1) < 1e-9


def test_variance_estimates_closed_form():
    # box values +-a with equal weight: <m> = 0, <m^2> = a^2, <|m|> = a
    a, Lb, kT, n = 0.01, 8, 2e-4, 1000
    est = M.hist_estimates(np.ones(12), 1.0, Lb, kT, n=n, sum_m=0.0, sum_m2=n * a * a, sum_abs_m=n * a)
    assert est["chi_var"] == pytest.approx(Lb ** 3 * a * a / kT, rel=1e-14)
    assert abs(est["chi_var_low"]) < 1e-9


def test_sampled_gaussian_estimators_agree():
    """Far above T_c the three estimates agree (Sec. IV C): sampled Gaussian
    box values, 4e6 of them.  With 101 bins over +-8 sigma the centre bin
    holds ~2.5e5 values (0.2% relative error, 0.4% on chi) and its bin
    averaging biases chi by 0.2%: agreement within 2.5%."""
    rng = np.random.default_rng(3)
    Lb, kT, chi = 2, 1e-4, 1.7
    sigma = math.sqrt(kT * chi / Lb ** 3)
    m = rng.normal(0.0, sigma, 4_000_000)
    h, bins = 8 * sigma, 101
    c = M.box_histogram(m, bins, h)
    assert c.sum() == m.size
    est = M.hist_estimates(c, h, Lb, kT, n=m.size, sum_m=m.sum(), sum_m2=(m * m).sum(), sum_abs_m=np.abs(m).sum())
    assert abs(est["chi_var"] / chi - 1) < 0.01
    assert abs(est["chi_center"] / est["chi_var"] - 1) < 0.025
    # the fullest bin of one Gaussian sits at its centre (within a few bins)
    assert est["m_max"] < 5 * (2 * h / bins)


def test_accumulator_histogram_counts_every_box():
    rng = np.random.default_rng(5)
    S = 8
    acc = M.Accumulator(S, hist_bins=16, hist_range=0.01)
    for _ in range(3):
        acc.add(1.0 + 1e-3 * rng.standard_normal(S ** 3))
    for L in acc.levels:
        assert acc.hist[L].sum() == 3 * (S // L) ** 3
    # a uniform field puts every box at m = 0: the bin [0, w)
    flat = M.Accumulator(S, hist_bins=16, hist_range=0.01)
    flat.add(np.full(S ** 3, 1.25))
    for L in flat.levels:
        assert flat.hist[L][8] == (S // L) ** 3


@pytest.mark.parametrize("w_over_s", [0.05, 0.1, 0.2])
def test_gauss_fit_recovers_chi_of_binned_gaussian(w_over_s):
    """Exact bin probabilities of a Gaussian: the fitted variance, with
    Sheppard's w^2/12 taken off, is the Gaussian's to O((w/s)^4); without
    the correction it would be off by (w/s)^2 / 12 (2e-4 to 3.3e-3)."""
    Lb, kT, chi = 4, 1e-4, 7.5
    sigma = math.sqrt(kT * chi / Lb ** 3)
    bins = 2 * int(round(5.0 / w_over_s)) + 1
    h = 0.5 * bins * w_over_s * sigma
    edges = np.linspace(-h, h, bins + 1)
    c = _counts_from_density(_gauss_bin_probs(edges, 0.0, sigma), 1e15)
    est = M.hist_estimates(c, h, Lb, kT, n=1.0, sum_m=0.0, sum_m2=sigma ** 2, sum_abs_m=0.0)
    assert abs(est["chi_fit"] / chi - 1) < 0.05 * w_over_s ** 2 / 12
    assert est["m_fit"] < 1e-6 * sigma


def test_gauss_fit_finds_an_off_centre_peak():
    """A peak centred 0.37 bin widths off a bin centre: the fit's centre is
    the Gaussian's, not the bin's."""
    Lb, kT, chi = 2, 1e-4, 2.0
    sigma = math.sqrt(kT * chi / Lb ** 3)
    bins, h = 400, 0.02
    w = 2 * h / bins
    mu = -h + (260 + 0.5) * w + 0.37 * w
    edges = np.linspace(-h, h, bins + 1)
    c = _counts_from_density(_gauss_bin_probs(edges, mu, sigma), 1e15)
    got_mu, s2 = M.gauss_fit_peak(c[:bins], h)
    assert abs(got_mu - mu) < 1e-4 * w
    assert abs(s2 / sigma ** 2 - 1) < 1e-4


def test_gauss_fit_two_peaks_with_interfacial_plateau():
    """Eq. (PL-lowT) plus a flat interfacial density between the peaks
    (1e-3 of the peak height, as in the coexistence regime, over
    |m| < M_L - 3 s): fitting the fullest peak recovers chi and M_L, while
    the peak height, normalised by every value, is biased by the plateau's
    share."""
    Lb, kT, chi, ML = 2, 1e-4, 3.0, 0.05
    sigma = math.sqrt(kT * chi / Lb ** 3)
    h, bins = 0.1, 1600
    edges = np.linspace(-h, h, bins + 1)
    p = 0.5 * (_gauss_bin_probs(edges, ML, sigma) + _gauss_bin_probs(edges, -ML, sigma))
    w = 2 * h / bins
    centres = edges[:-1] + 0.5 * w
    plateau = np.where(np.abs(centres) < ML - 3 * sigma, 1e-3 * p.max(), 0.0)
    c = _counts_from_density(p + plateau, 1e15)
    est = M.hist_estimates(c, h, Lb, kT, n=1.0, sum_m=0.0, sum_m2=ML ** 2 + sigma ** 2, sum_abs_m=ML)
    assert abs(est["m_fit"] - ML) < 1e-3 * w
    assert abs(est["chi_fit"] / chi - 1) < 1e-3
    share = plateau.sum() / (p + plateau).sum()
    assert abs(est["chi_peak"] / chi - (1 + share) ** 2) < 2e-3


def test_gauss_fit_of_sampled_gaussian():
    """Sampled values (Poisson counts): the count-weighted fit recovers chi
    within its statistical error (4e6 values, ~30 bins in the window:
    about 0.1% on s^2; tolerance 1%)."""
    rng = np.random.default_rng(11)
    Lb, kT, chi = 2, 1e-4, 1.7
    sigma = math.sqrt(kT * chi / Lb ** 3)
    m = rng.normal(0.3 * sigma, sigma, 4_000_000)
    h, bins = 8 * sigma, 121
    c = M.box_histogram(m, bins, h)
    est = M.hist_estimates(c, h, Lb, kT, n=m.size, sum_m=m.sum(), sum_m2=(m * m).sum(), sum_abs_m=np.abs(m).sum())
    assert abs(est["chi_fit"] / chi - 1) < 0.01
    assert abs(est["m_fit"] - 0.3 * sigma) < 0.01 * sigma


def test_gauss_fit_degenerate_cases():
    """One filled bin (fewer than three in the window) and a histogram
    rising towards its edges (no peak: curvature not negative) have no fit."""
    one = np.zeros(12)
    one[5] = 1000
    mu, s2 = M.gauss_fit_peak(one, 1.0)
    assert math.isnan(mu) and math.isnan(s2)
    u = np.arange(20) - 9.5
    cup = np.rint(1000 * np.exp(0.01 * u * u))
    mu, s2 = M.gauss_fit_peak(cup, 1.0)
    assert math.isnan(s2)
    est = M.hist_estimates(np.concatenate([one, [0, 0]]), 1.0, 2, 1e-4, 1.0, 0.0, 1e-4, 0.0)
    assert math.isnan(est["chi_fit"])
