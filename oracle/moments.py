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
  here evaluated along the three lattice axes, k_m = 2 pi m / S,
  1 <= m < S/2 (k = 0 vanishes by mass conservation; the zone-edge mode is
  excluded).

Arrays are flat, site = x + S*(y + S*z); reshaped to [z, y, x].
"""
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

    return {"P0": P0, "chi_center": ratio(vol, 2.0 * np.pi * kT * P0 ** 2),
            "m_max": m_max, "P_max": Pmax, "chi_peak": ratio(vol, 8.0 * np.pi * kT * Pmax ** 2),
            "chi_var": ratio(vol * (mean2 - mean ** 2), kT), "chi_var_low": ratio(vol * (mean2 - mabs ** 2), kT)}


class Accumulator:
    """Sums of the block moments and axis structure factor over samples, the
    way the GPU library accumulates them; with ``hist_bins`` > 0 also the
    histogram of every level over [-hist_range, hist_range)."""

    def __init__(self, S, n_levels=0, hist_bins=0, hist_range=0.0):
        self.S = S
        self.levels = levels(S, n_levels)
        self.n_samples = 0
        self.sums = {L: {k: 0.0 for k in ("n",) + MOMENT_KEYS} for L in self.levels}
        self.sk = np.zeros((3, max(S // 2 - 1, 0)))
        self.series = []
        self.hist_bins, self.hist_range = hist_bins, hist_range
        self.hist = {L: np.zeros(hist_bins + 2, dtype=np.int64) for L in self.levels} if hist_bins else {}

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
