"""Observables of the finite-size-scaling analysis, written as plain definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

- Order parameter, Sec. II A, Eq. (op): phi = (rho - rho0)/rho0 with rho0 the
  global mean density.
- Block order parameter, Sec. II B, Eq. (mL): m_L^(b) = L^-d sum_{i in b} phi_i
  over the sub-boxes b of edge L = S/2^l that tile the lattice; the moments of
  m_L feed Eqs. (ML), (chiL), (chiL-lowT).  E_L^(b) = (2 L^d)^-1 sum phi_i^2
  feeds Eq. (CL).
- Order-parameter distribution, Sec. II C: P_L(m) is the histogram of the
  box values m_L^(b) over all boxes and samples (Eq. (PL-def)); susceptibility
  estimates from its central height (Eq. (PL-highT) at m = 0), from the height
  of its maximum (Eq. (PL-lowT) at m = M_L, Sec. IV C) and from its variance
  (Eqs. (chiL), (chiL-lowT)).
- Structure factor, Sec. IV A, Eq. (G-comput): C(k) = N^-1 |sum_r phi e^{-ik.r}|^2,
  evaluated along the three lattice axes, k_m = 2 pi m / S, 1 <= m < S/2
  (k = 0 vanishes by mass conservation; the zone-edge mode is excluded), and
  over the whole lattice (three-dimensional FFT), averaged over shells of
  |m| for the Ornstein-Zernike fit of Eq. (CMF) (Sec. IV A).

Arrays are flat, site = x + S*(y + S*z); reshaped to [z, y, x].
"""
import math

import numpy as np

MOMENT_KEYS = ("m", "m2", "m3", "m4", "abs_m", "E", "E2")


def levels(S, n_levels=0):
    """Block edges L_b = S / 2^l, l = 1, 2, ..., while S / 2^l is an integer
    (at most ``n_levels`` of them if n_levels > 0)."""
    out = []
    L = S
    while L % 2 == 0 and L // 2 >= 1:
        L //= 2
        out.append(L)
        if n_levels and len(out) == n_levels:
            break
    return out


def order_parameter(rho):
    rho = np.asarray(rho, dtype=np.float64)
    rho0 = rho.mean()
    return (rho - rho0) / rho0


def block_values(phi, S, L):
    """m_L and E_L of every box of edge L (one value per box)."""
    p = np.asarray(phi, dtype=np.float64).reshape(S, S, S)
    nb = S // L
    blocks = p.reshape(nb, L, nb, L, nb, L)
    m = blocks.sum(axis=(1, 3, 5)) / L ** 3
    E = (blocks ** 2).sum(axis=(1, 3, 5)) / (2.0 * L ** 3)
    return m.reshape(-1), E.reshape(-1)


def block_sums(phi, S, L):
    """Sums over boxes of m, m^2, m^3, m^4, |m|, E, E^2 and the box count."""
    m, E = block_values(phi, S, L)
    return {"n": m.size, "m": m.sum(), "m2": (m ** 2).sum(), "m3": (m ** 3).sum(),
            "m4": (m ** 4).sum(), "abs_m": np.abs(m).sum(), "E": E.sum(), "E2": (E ** 2).sum()}


def axis_structure_factor(phi, S):
    """S_alpha(k_m), alpha = x, y, z (rows), m = 1 .. S/2 - 1 (columns)."""
    p = np.asarray(phi, dtype=np.float64).reshape(S, S, S)   # [z, y, x]
    planes = [p.sum(axis=(0, 1)), p.sum(axis=(0, 2)), p.sum(axis=(1, 2))]  # P_x, P_y, P_z
    n = np.arange(S)
    ms = np.arange(1, S // 2)
    E = np.exp(-2j * np.pi * np.outer(ms, n) / S)
    return np.array([np.abs(E @ P) ** 2 / S ** 3 for P in planes])


def structure_factor_3d(phi, S):
    """C(k) = N^-1 |sum_r phi(r) e^{-i k.r}|^2 at every k = 2 pi m / S, as an
    [mz, my, mx] array (Eq. (G-comput)); the library FFT is the DFT."""
    p = np.asarray(phi, dtype=np.float64).reshape(S, S, S)
    return np.abs(np.fft.fftn(p)) ** 2 / S ** 3


def folded_modes(S):
    """Integer wave numbers m in (-S/2, S/2] of the FFT index order."""
    i = np.arange(S)
    return np.where(i <= S // 2, i, i - S)


def lattice_laplacian_symbol(kx, ky, kz):
    """-(discrete Laplacian) in Fourier space for the isotropic D3Q19 stencil
    6 sum_i w_i (1 - cos k.c_i): ~k^2 at small k (the lattice k^2 of Eq. (CMF),
    Sec. IV A)."""
    axis = 2 * (3 - np.cos(kx) - np.cos(ky) - np.cos(kz)) / 3.0
    diag = (12 - 2 * (np.cos(kx + ky) + np.cos(kx - ky) + np.cos(ky + kz) + np.cos(ky - kz)
                      + np.cos(kz + kx) + np.cos(kz - kx))) / 6.0
    return axis + diag


def shells(S):
    """Shell of every mode (array [mz, my, mx]): s = floor(|m| + 1/2) with m
    folded into (-S/2, S/2]; the k = 0 mode is shell 0 and is excluded from
    every shell average.  Returns (shell index array, number of shells incl. 0)."""
    m = folded_modes(S).astype(np.float64)
    mz, my, mx = np.meshgrid(m, m, m, indexing="ij")
    r = np.sqrt(mx * mx + my * my + mz * mz)
    sh = np.floor(r + 0.5).astype(np.int64)
    return sh, int(sh.max()) + 1


def shell_average(C, S):
    """Per shell s >= 1: number of modes, sum of C, mean k^2 (continuum,
    k = 2 pi m / S) and mean lattice Laplacian symbol over its modes."""
    sh, ns = shells(S)
    m = folded_modes(S) * (2 * np.pi / S)
    kz, ky, kx = np.meshgrid(m, m, m, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    lap = lattice_laplacian_symbol(kx, ky, kz)
    out = {"modes": np.zeros(ns, dtype=np.int64), "sum_C": np.zeros(ns), "k2": np.zeros(ns), "lap": np.zeros(ns)}
    flat = sh.reshape(-1)
    live = flat > 0
    out["modes"] = np.bincount(flat[live], minlength=ns)
    out["sum_C"] = np.bincount(flat[live], weights=np.asarray(C).reshape(-1)[live], minlength=ns)
    with np.errstate(invalid="ignore", divide="ignore"):
        out["k2"] = np.bincount(flat[live], weights=k2.reshape(-1)[live], minlength=ns) / out["modes"]
        out["lap"] = np.bincount(flat[live], weights=lap.reshape(-1)[live], minlength=ns) / out["modes"]
    return out


def oz_fit(mean_C, modes, x, kT, use):
    """Ornstein-Zernike fit, Eq. (CMF): C = kT chi / (1 + xi^2 k^2), i.e.
    1/C = A + B x with A = 1/(kT chi), B = xi^2 A, x the shell's k^2 (or the
    lattice Laplacian symbol).  Weighted least squares over the shells
    selected by ``use``, weight modes * C^2 (the inverse variance of 1/C for
    a shell mean of `modes` exponentially distributed mode values).
    Returns chi, xi (nan if B/A < 0), C0 = 1/A, A, B."""
    y = 1.0 / np.asarray(mean_C, dtype=np.float64)[use]
    xx = np.asarray(x, dtype=np.float64)[use]
    w = np.asarray(modes, dtype=np.float64)[use] * np.asarray(mean_C, dtype=np.float64)[use] ** 2
    S0, S1, S2 = w.sum(), (w * xx).sum(), (w * xx * xx).sum()
    T0, T1 = (w * y).sum(), (w * xx * y).sum()
    det = S0 * S2 - S1 * S1
    A = (S2 * T0 - S1 * T1) / det
    B = (S0 * T1 - S1 * T0) / det
    xi = np.sqrt(B / A) if B / A >= 0 else float("nan")
    return {"chi": 1.0 / (kT * A), "xi": xi, "C0": 1.0 / A, "A": A, "B": B}


def box_histogram(m, bins, h):
    """Counts of box values m over ``bins`` equal bins covering [-h, h): the
    value goes to bin k = floor((m + h) * (bins / (2 h))) when 0 <= k < bins.
    Returns bins + 2 integers: the bins, then the count of values below -h,
    then the count of values at or above h (those outside the bins)."""
    m = np.asarray(m, dtype=np.float64).reshape(-1)
    inv_w = bins / (2.0 * h)
    k = np.floor((m + h) * inv_w)
    out = np.zeros(bins + 2, dtype=np.int64)
    inside = (k >= 0) & (k < bins)
    np.add.at(out, k[inside].astype(np.int64), 1)
    out[bins] = np.count_nonzero(k < 0)
    out[bins + 1] = np.count_nonzero(k >= bins)
    return out


def hist_estimates(counts, h, Lb, kT, n, sum_m, sum_m2, sum_abs_m, d=3):
    """Susceptibility estimates of one block level from its histogram
    ``counts`` (layout of box_histogram) and its moment sums over ``n`` box
    values, Sec. II B-C and IV C:
      P(k)       = counts_k / (n_total w), the density of bin k (w = 2h/bins,
                   n_total = every counted value, the outside ones included)
      P0         = density at m = 0: the bin holding 0 (odd bins) or the mean
                   of the two bins that meet at 0 (even bins)
      chi_center = L^d / (2 pi kT P0^2)            Eq. (PL-highT) at m = 0
      m_max      = |centre| of the fullest bin (lowest index on ties), M_L
                   taken as the position of the maximum of P_L
      chi_peak   = L^d / (8 pi kT P(m_max)^2)      Eq. (PL-lowT) at m = M_L,
                   the other Gaussian neglected
      chi_var    = L^d (<m^2> - <m>^2) / kT        Eq. (chiL)
      chi_var_low = L^d (<m^2> - <|m|>^2) / kT     Eq. (chiL-lowT)
      m_fit, chi_fit  a Gaussian fitted to the fullest peak (gauss_fit_peak):
                   |its centre| and L^d s^2 / kT
    A zero denominator (an empty bin, kT = 0) gives +inf."""
    counts = np.asarray(counts, dtype=np.float64)
    bins = counts.size - 2
    w = 2.0 * h / bins
    total = counts.sum()
    dens = counts[:bins] / (total * w)
    if bins % 2:
        P0 = dens[bins // 2]
    else:
        P0 = 0.5 * (dens[bins // 2 - 1] + dens[bins // 2])
    kmax = int(np.argmax(counts[:bins]))
    m_max = abs(-h + (kmax + 0.5) * w)
    Pmax = dens[kmax]
    vol = float(Lb) ** d
    mean, mean2, mabs = sum_m / n, sum_m2 / n, sum_abs_m / n

    def ratio(num, den):  # an empty centre (den = 0) gives an infinite estimate
        return num / den if den > 0 else float("inf")

    mu, s2 = gauss_fit_peak(counts[:bins], h)
    chi_fit = ratio(vol * s2, kT) if np.isfinite(s2) else float("nan")
    return {"P0": P0, "chi_center": ratio(vol, 2.0 * np.pi * kT * P0 ** 2),
            "m_max": m_max, "P_max": Pmax, "chi_peak": ratio(vol, 8.0 * np.pi * kT * Pmax ** 2),
            "chi_var": ratio(vol * (mean2 - mean ** 2), kT), "chi_var_low": ratio(vol * (mean2 - mabs ** 2), kT),
            "m_fit": abs(mu), "chi_fit": chi_fit}


FIT_LEVEL = math.exp(-2.0)   # window edge: a Gaussian falls to this at +-2 s


def gauss_fit_peak(counts, h):
    """A Gaussian fitted to the fullest peak of a histogram (the in-range
    bins of box_histogram over [-h, h)), Sec. IV C: the contiguous bins
    around the fullest one (lowest index on ties) that hold at least
    exp(-2) of its count (about +-2 standard deviations, so the region
    between two peaks stays out) give ln(count) = c0 + c1 u + c2 u^2 by
    least squares weighted with the counts (the inverse variance of ln of a
    Poisson count), u = bin index - fullest index.  Centre mu = centre of
    the fullest bin - w c1 / (2 c2); variance s^2 = -w^2 / (2 c2) - w^2 / 12,
    the last term Sheppard's correction for counts grouped in bins of width
    w.  Returns (mu, s^2), or (nan, nan) when fewer than three bins qualify
    or the fitted curvature is not negative."""
    c = np.asarray(counts, dtype=np.float64)
    bins = c.size
    w = 2.0 * h / bins
    k0 = int(np.argmax(c))
    thr = c[k0] * FIT_LEVEL
    lo = k0
    while lo > 0 and c[lo - 1] >= thr:
        lo -= 1
    hi = k0
    while hi < bins - 1 and c[hi + 1] >= thr:
        hi += 1
    if hi - lo + 1 < 3:
        return float("nan"), float("nan")
    u = np.arange(lo, hi + 1, dtype=np.float64) - k0
    sw = np.sqrt(c[lo:hi + 1])
    A = np.stack([np.ones_like(u), u, u * u], axis=1) * sw[:, None]
    coef = np.linalg.lstsq(A, np.log(c[lo:hi + 1]) * sw, rcond=None)[0]
    if not coef[2] < 0:
        return float("nan"), float("nan")
    mu = -h + (k0 + 0.5) * w - w * coef[1] / (2.0 * coef[2])
    return mu, -w * w / (2.0 * coef[2]) - w * w / 12.0


class Accumulator:
    """Sums of the block moments and axis structure factor over samples, the
    way the GPU library accumulates them; with ``hist_bins`` > 0 also the
    histogram of every level over [-hist_range, hist_range)."""

    def __init__(self, S, n_levels=0, hist_bins=0, hist_range=0.0, sk3=False):
        self.S = S
        self.levels = levels(S, n_levels)
        self.n_samples = 0
        self.sums = {L: {k: 0.0 for k in ("n",) + MOMENT_KEYS} for L in self.levels}
        self.sk = np.zeros((3, max(S // 2 - 1, 0)))
        self.series = []
        self.hist_bins, self.hist_range = hist_bins, hist_range
        self.hist = {L: np.zeros(hist_bins + 2, dtype=np.int64) for L in self.levels} if hist_bins else {}
        self.sk3 = np.zeros(shells(S)[1]) if sk3 else None
        self.n_sk3 = 0

    def add_sk3(self, rho):
        """Shell sums of the 3D structure factor of one sample."""
        self.sk3 += shell_average(structure_factor_3d(order_parameter(rho), self.S), self.S)["sum_C"]
        self.n_sk3 += 1

    def add(self, rho, step=None, j=None):
        phi = order_parameter(rho)
        rec = {"step": step, "mass": float(np.sum(rho))}
        if j is not None:
            rec["momentum"] = np.asarray(j).reshape(3, -1).sum(axis=1)
        for L in self.levels:
            bs = block_sums(phi, self.S, L)
            for k, v in bs.items():
                self.sums[L][k] += v
            rec[L] = {k: bs[k] / bs["n"] for k in MOMENT_KEYS}
            if self.hist_bins:
                self.hist[L] += box_histogram(block_values(phi, self.S, L)[0], self.hist_bins, self.hist_range)
        if self.S >= 4:
            self.sk += axis_structure_factor(phi, self.S)
        self.n_samples += 1
        self.series.append(rec)


def binder(m2, m4):
    """U_L = 1 - <m^4> / (3 <m^2>^2) (fourth-order cumulant of the block order
    parameter; zero for a Gaussian distribution)."""
    return 1.0 - m4 / (3.0 * m2 ** 2)
