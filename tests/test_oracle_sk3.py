"""Pins of the oracle's three-dimensional structure factor, its shell
averages and the Ornstein-Zernike fit (Sec. IV A, Eqs. (G-comput), (CMF))."""
import math

import numpy as np
import pytest

from oracle import moments as M

C19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
       (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
W19 = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12


def test_fft_equals_brute_force_dft():
    rng = np.random.default_rng(1)
    S = 4
    phi = rng.standard_normal(S ** 3)
    C = M.structure_factor_3d(phi, S)
    p = phi.reshape(S, S, S)   # [z, y, x]
    r = np.arange(S)
    for mz in range(S):
        for my in range(S):
            for mx in range(S):
                acc = 0j
                for z in r:
                    for y in r:
                        for x in r:
                            acc += p[z, y, x] * np.exp(-2j * np.pi * (mx * x + my * y + mz * z) / S)
                assert abs(abs(acc) ** 2 / S ** 3 - C[mz, my, mx]) < 1e-12


def test_single_plane_wave():
    """phi = cos(2 pi m.r / S): C = N/4 at +-m, zero elsewhere."""
    S = 8
    z, y, x = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    m = (1, 2, 3)
    phi = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / S)
    C = M.structure_factor_3d(phi.reshape(-1), S)
    N = S ** 3
    assert abs(C[m[2], m[1], m[0]] - N / 4) < 1e-9
    assert abs(C[-m[2], -m[1], -m[0]] - N / 4) < 1e-9
    assert abs(C.sum() - N / 2) < 1e-9
    # it lands in shell floor(sqrt(14) + 1/2) = 4
    sa = M.shell_average(C, S)
    assert abs(sa["sum_C"][4] - N / 2) < 1e-9 and abs(sa["sum_C"].sum() - N / 2) < 1e-9


@pytest.mark.parametrize("S", [4, 6, 7, 8, 12])
def test_shell_counts_by_enumeration(S):
    counts = {}
    half = S // 2
    for a in range(S):
        for b in range(S):
            for c in range(S):
                v = [t if t <= half else t - S for t in (a, b, c)]
                r = math.sqrt(sum(t * t for t in v))
                s = int(math.floor(r + 0.5))
                counts[s] = counts.get(s, 0) + 1
    sa = M.shell_average(np.zeros((S, S, S)), S)
    assert sa["modes"][0] == 0
    for s_, n in counts.items():
        if s_ > 0:
            assert sa["modes"][s_] == n
    assert sa["modes"].sum() == S ** 3 - 1


def test_laplacian_symbol_is_the_stencil_eigenvalue():
    """The symbol is what the isotropic stencil 6 sum w_i [psi(x + c_i) - psi(x)]
    does to a plane wave (applied here with np.roll), and ~k^2 at small k."""
    S = 8
    z, y, x = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    for m in [(1, 0, 0), (1, 1, 0), (2, 1, 3), (4, 4, 4)]:
        k = [2 * np.pi * t / S for t in m]
        psi = np.cos(k[0] * x + k[1] * y + k[2] * z)
        lap = sum(6 * w * (np.roll(psi, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2)) - psi) for w, c in zip(W19, C19))
        val = M.lattice_laplacian_symbol(*k)
        assert np.allclose(lap, -val * psi, atol=1e-12)
    kk = 1e-3
    assert abs(M.lattice_laplacian_symbol(kk, 0.5 * kk, 0.2 * kk) / (kk * kk * 1.29) - 1) < 1e-5


def test_oz_fit_recovers_parameters():
    kT, chi, xi = 1e-4, 20.0, 1.9
    S = 16
    sa = M.shell_average(np.zeros((S, S, S)), S)
    use = (sa["modes"] > 0) & (np.sqrt(sa["k2"]) < 1.2)
    use[0] = False
    meanC = np.where(sa["modes"] > 0, kT * chi / (1 + xi * xi * sa["k2"]), 1.0)
    fit = M.oz_fit(meanC, sa["modes"], sa["k2"], kT, use)
    assert abs(fit["chi"] / chi - 1) < 1e-12 and abs(fit["xi"] / xi - 1) < 1e-12
    # a wrong-curvature data set gives no real xi
    bad = np.where(sa["modes"] > 0, kT * chi * (1 + 0.1 * sa["k2"]), 1.0)
    assert math.isnan(M.oz_fit(bad, sa["modes"], sa["k2"], kT, use)["xi"])


def test_axis_modes_of_3d_match_axis_structure_factor():
    rng = np.random.default_rng(4)
    S = 8
    phi = rng.standard_normal(S ** 3)
    C = M.structure_factor_3d(phi, S)
    ax = M.axis_structure_factor(phi, S)  # rows x, y, z over m = 1..S/2-1
    # the axis structure factor is the 3D one on the axes: S_x(m) = C at (m, 0, 0)
    for mi in range(1, S // 2):
        assert abs(ax[0, mi - 1] - C[0, 0, mi]) < 1e-10
        assert abs(ax[1, mi - 1] - C[0, mi, 0]) < 1e-10
        assert abs(ax[2, mi - 1] - C[mi, 0, 0]) < 1e-10
