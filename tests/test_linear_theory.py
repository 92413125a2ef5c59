"""Pins of the linearized theory itself (it is used to pin the oracle's and
the GPU's long-run statistics)."""
import numpy as np
import pytest

import linear_theory as lt


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_ideal_gas_equipartition_exact(tau):
    """Without the force the lattice gas has S(k) = rho0 kT / c_s^2 and
    <|j_a(k)|^2>/N = rho0 kT at every wave vector (Eq. (vel-correl))."""
    kT, rho0 = 1e-4, 1.3
    for k in [(0.3, 0, 0), (1.0, 0.4, -0.2), (2.9, 2.0, 1.1)]:
        s = lt.structure_factor(k, tau, kT=kT, rho0=rho0, force_off=True)
        assert abs(s / (3 * rho0 * kT) - 1) < 1e-10
        jv = lt.momentum_variance(k, tau, kT=kT, rho0=rho0, force_off=True)
        assert np.allclose(jv / (rho0 * kT), 1, atol=1e-10)


def test_ornstein_zernike_limit():
    """With the force and b = 0, S(k) -> kT / (a + kappa_eff k^2) at small k
    (Sec. II A, Eq. (CMF)); the lattice shifts kappa by 1/12 independently of
    tau and kappa."""
    kT = 1e-4
    for tau in (0.8, 1.0, 1.5):
        for a, kappa in ((0.05, 0.1), (0.2, 0.0), (0.01, 0.5)):
            for q in (1e-3, 1e-2):
                s = lt.structure_factor((q, 0, 0), tau, a=a, kappa=kappa, kT=kT)
                assert abs(s * (a + (kappa + 1 / 12) * q * q) / kT - 1) < 2e-5 + 0.05 * q ** 2 / a
    # isotropy of the small-k limit
    q = 0.01
    s1 = lt.structure_factor((q, 0, 0), 1.0, a=0.05, kappa=0.1, kT=kT)
    s2 = lt.structure_factor((q / np.sqrt(3),) * 3, 1.0, a=0.05, kappa=0.1, kT=kT)
    assert abs(s1 / s2 - 1) < 1e-6


def test_zone_edge_frozen():
    """The k = (pi, 0, 0) mode has a unit-modulus eigenvalue: no stationary
    state is defined there, and it is excluded from the comparisons."""
    assert lt.structure_factor((np.pi, 0, 0), 1.0, force_off=True, kT=1e-4) is None


def test_moment_projectors_are_complete():
    E = lt.basis()
    Nrm = (E * E * lt.W).sum(axis=1)
    total = sum(lt.W[:, None] * np.outer(E[a], E[a]) / Nrm[a] for a in range(19))
    assert np.allclose(total, np.eye(19), atol=1e-14)


@pytest.mark.parametrize("tau,tb,tg", [(0.8, 1.3, 0.6), (1.0, 0.55, 1.9), (1.4, 1.0, 1.0)])
def test_ideal_gas_equipartition_separate_rates(tau, tb, tg):
    """Every non-conserved moment relaxes with its own gamma_a and receives
    noise of variance proportional to 1 - gamma_a^2: the ideal gas keeps
    S(k) = 3 rho0 kT and <|j_a(k)|^2>/N = rho0 kT at every k for any rates."""
    kT, rho0 = 1e-4, 1.1
    for k in [(0.3, 0, 0), (1.0, 0.4, -0.2), (2.9, 2.0, 1.1)]:
        s = lt.structure_factor(k, tau, kT=kT, rho0=rho0, force_off=True, tau_bulk=tb, tau_ghost=tg)
        assert abs(s / (3 * rho0 * kT) - 1) < 1e-10
        jv = lt.momentum_variance(k, tau, kT=kT, rho0=rho0, force_off=True, tau_bulk=tb, tau_ghost=tg)
        assert np.allclose(jv / (rho0 * kT), 1, atol=1e-10)
