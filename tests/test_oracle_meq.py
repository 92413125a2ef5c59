"""Pins of the oracle of the paper's model on D3Q19 (oracle/d3q19_meq.py):
the noise covariance construction against the matrix the paper prints for
D2Q9, the closed-form D3Q19 factor against the construction, the
equilibrium against Eq. (holdych-cond) and the standard equilibrium, exact
conservation, and equilibrium statistics."""
import os

import numpy as np
import pytest

from oracle import d2q9 as D2
from oracle import d3q19_meq as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_lbnoise_d2q9_matrix.txt")


def _printed_d2q9(x):
    with open(GOLDEN) as fh:
        ent = [tuple(float(v) for v in line.split()) for line in fh if line.strip() and not line.startswith("#")]
    Mp = np.zeros((6, 6))
    for r, c, c0, c1 in ent:
        Mp[int(r) - 3, int(c) - 3] = Mp[int(c) - 3, int(r) - 3] = c0 + c1 * x
    return Mp


@pytest.mark.parametrize("x", [-0.3, 0.0, 0.01, 0.2, 1 / 3, 0.5, 0.59])
def test_construction_reproduces_the_papers_d2q9_matrix(x):
    """The construction applied to D2Q9 (its velocities, weights, basis and
    an equilibrium with the pressure on the moving populations) gives the
    printed matrix of Eq. (lbnoise) on the non-conserved moments, at every
    c_s^2, and zero rows on the conserved ones."""
    if x == 0.0:
        x = 1e-9  # the rest population's variance rho kT / c_s^2 diverges at 0
    Mc = M.fdt_moment_covariance(D2.C, D2.W, D2.E, x)
    assert np.allclose(Mc[3:, 3:], _printed_d2q9(x), atol=1e-9 * max(1.0, 1.0 / x), rtol=0)
    assert np.abs(Mc[:3]).max() < 1e-12 * max(1.0, 1.0 / x)


@pytest.mark.parametrize("x", [-0.2, 0.02, 0.2, 1 / 3, 0.45])
def test_d3q19_factor_is_the_construction(x):
    Mc = M.fdt_moment_covariance(M.C, M.W, M.E, x)
    assert np.abs(Mc[:4]).max() < 1e-12 * max(1.0, 1.0 / abs(x))
    L44, L164, L1616 = M.noise_factor(x)
    blk = np.array([[L44 * L44, L44 * L164], [L44 * L164, L164 * L164 + L1616 * L1616]])
    assert np.allclose(blk, Mc[np.ix_([4, 16], [4, 16])], atol=1e-12)
    rest = [a for a in range(4, 19) if a not in (4, 16)]
    assert np.allclose(Mc[np.ix_(rest, rest)], np.diag(M.NORM[rest]), atol=1e-12)
    assert np.abs(Mc[np.ix_([4, 16], rest)]).max() < 1e-12
    # at the lattice sound speed the covariance is the basis norms
    if x == 1 / 3:
        assert abs(L164) < 1e-15 and np.isclose(L44 ** 2, M.NORM[4]) and np.isclose(L1616 ** 2, M.NORM[16])


def _random_fields(n, rng):
    rho = 1.0 + 0.05 * rng.standard_normal(n)
    j = 0.02 * rng.standard_normal((3, n))
    grad = 0.1 * rng.standard_normal((3, n))
    lap = 0.1 * rng.standard_normal(n)
    return rho, j, grad, lap


def test_equilibrium_moments_are_holdych_condition():
    """Sum f = rho, sum c f = j, sum c c f = Pi (Eq. (holdych-cond) with
    Eq. (press-th)), on random fields with every term switched on."""
    rng = np.random.default_rng(1)
    rho, j, grad, lap = _random_fields(50, rng)
    prm = dict(a=0.03, b=0.7, kappa=0.2, rho_c=1.0, tau=0.8)
    f = M.equilibrium(rho, j, grad, lap, prm)
    p_iso, Pi = M.second_moment(rho, j, grad, lap, prm)
    c = M.C.astype(float)
    assert np.allclose(f.sum(axis=0), rho, atol=1e-14, rtol=0)
    assert np.allclose(c.T @ f, j, atol=1e-14, rtol=0)
    assert np.allclose(np.einsum("ia,ib,in->abn", c, c, f), Pi, atol=1e-14, rtol=0)
    # Pi itself, written out from Eq. (press-th) and Eq. (holdych-cond)
    p0, _ = M.thermo(rho, 0.03, 0.7, 1.0)
    u = j / rho
    nu = (0.8 - 0.5) / 3
    k = 5
    P = (p0[k] - 0.2 * rho[k] * lap[k] - 0.1 * grad[:, k] @ grad[:, k]) * np.eye(3) + 0.2 * np.outer(grad[:, k], grad[:, k])
    want = P + rho[k] * np.outer(u[:, k], u[:, k]) + nu * (np.outer(u[:, k], grad[:, k]) + np.outer(grad[:, k], u[:, k])
                                                          + (u[:, k] @ grad[:, k]) * np.eye(3))
    assert np.allclose(Pi[:, :, k], want, atol=1e-15)


def test_ideal_gas_equilibrium_is_the_standard_one():
    rng = np.random.default_rng(2)
    rho = 1.0 + 0.05 * rng.standard_normal(40)
    u = 0.05 * rng.standard_normal((3, 40))
    Pi = rho / 3 * np.eye(3)[:, :, None] + rho * np.einsum("an,bn->abn", u, u)
    f = M.equilibrium_from(rho, rho * u, rho / 3, Pi)
    cu = M.C.astype(float) @ u
    std = M.W[:, None] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u * u).sum(axis=0))
    assert np.allclose(f, std, atol=1e-15, rtol=0)


def test_equilibrium_moments_closed_form():
    """The moments of the equilibrium in the basis, derived by hand:
    rho, j, tr Pi - rho, 3 Pi_xx - tr Pi, Pi_yy - Pi_zz, Pi_xy, Pi_yz,
    Pi_zx, zero third-order ghosts, rho - 3 p_iso, and zero anisotropic
    fourth-order ghosts (the GPU kernel uses this form)."""
    rng = np.random.default_rng(3)
    rho, j, grad, lap = _random_fields(30, rng)
    prm = dict(a=-0.02, b=1.5, kappa=0.1, rho_c=1.0, tau=1.3)
    m = M.E @ M.equilibrium(rho, j, grad, lap, prm)
    p_iso, Pi = M.second_moment(rho, j, grad, lap, prm)
    tr = Pi[0, 0] + Pi[1, 1] + Pi[2, 2]
    z = np.zeros_like(rho)
    want = np.array([rho, j[0], j[1], j[2], tr - rho, 3 * Pi[0, 0] - tr, Pi[1, 1] - Pi[2, 2],
                     Pi[0, 1], Pi[1, 2], Pi[2, 0], z, z, z, z, z, z, rho - 3 * p_iso, z, z])
    assert np.allclose(m, want, atol=1e-14, rtol=0)


def test_exact_conservation_with_the_quartic_term():
    """Mass and momentum are conserved to rounding for b > 0 (the property
    the force scheme lacks), with noise."""
    L = 6
    sim = M.Sim(L, 11, a=0.02, b=2.0, kappa=0.1, kT=1e-4, tau=0.8, init_sigma=0.02)
    rho0, j0 = sim.fields()
    sim.step(12)
    rho1, j1 = sim.fields()
    assert abs(rho1.sum() - rho0.sum()) < 1e-12 * rho0.sum()
    assert np.abs(j1.sum(axis=1) - j0.sum(axis=1)).max() < 1e-13


def test_equilibrium_statistics_8():
    """b = 0, a = 0.05, small kappa: density and momentum fluctuations
    equilibrate to <|rho_k|^2>/N = rho kT / c_s^2 = kT / a at the smallest
    k (Sec. III A: the compressibility of the Landau free energy) and
    <|j_k|^2>/N = rho kT per component at every k (equipartition,
    Eq. (vel-correl)).  8^3, 4000 steps after 1000, tolerance 6% (a few
    thousand correlated samples)."""
    L = 8
    prm = dict(a=0.05, b=0.0, kappa=1e-3, kT=1e-4, tau=0.8, init_sigma=0.0)
    sim = M.Sim(L, 5, **prm)
    sim.step(1000)
    S = np.zeros((L, L, L))
    J = np.zeros((L, L, L))
    n = 0
    for _ in range(800):
        sim.step(5)
        rho, j = sim.fields()
        rk = np.fft.fftn((rho - rho.mean()).reshape(L, L, L))
        S += np.abs(rk) ** 2 / L ** 3
        for a in range(3):
            J += np.abs(np.fft.fftn(j[a].reshape(L, L, L))) ** 2 / L ** 3 / 3
        n += 1
    S /= n
    J /= n
    kT, a = prm["kT"], prm["a"]
    smallest = [S[1, 0, 0], S[0, 1, 0], S[0, 0, 1]]
    lam = 6 * np.sum(M.W * (1 - np.cos(2 * np.pi / L * M.C[:, 0])))  # lattice k^2 of the smallest mode
    want = kT / (a + prm["kappa"] * lam)
    assert abs(np.mean(smallest) / want - 1) < 0.06
    Jm = J.copy()
    Jm[0, 0, 0] = np.nan  # total momentum is conserved
    assert abs(np.nanmean(Jm) / kT - 1) < 0.03
