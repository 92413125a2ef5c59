"""Pins of the oracle's difference operators, chemical potential and force.

Plane-wave symbols below were derived by hand from the D3Q19 weights (not by
evaluating the stencil): for psi = cos(k . r)
  k = (q, 0, 0):  lap psi = -2 (1 - cos q) psi,
                  grad_x psi = -sin q sin(k . r)
  k = (q, q, 0):  lap psi = -[8/3 (1 - cos q) + 1/3 (1 - cos 2q)] psi,
                  grad_x psi = grad_y psi = -[2/3 sin q + 1/6 sin 2q] sin(k . r)
  k = (q, q, q):  lap psi = -[2 (1 - cos q) + (1 - cos 2q)] psi,
                  grad_a psi = -[1/3 sin q + 1/3 sin 2q] sin(k . r)
All reduce to -|k|^2 and -k at small q."""
import numpy as np
import pytest

import oracle

S = 8


def coords(S):
    z, y, x = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


CASES = [
    ((1, 0, 0), lambda q: 2 * (1 - np.cos(q)), lambda q: (np.sin(q), 0.0, 0.0)),
    ((1, 1, 0), lambda q: 8 / 3 * (1 - np.cos(q)) + (1 - np.cos(2 * q)) / 3,
     lambda q: (2 / 3 * np.sin(q) + np.sin(2 * q) / 6,) * 2 + (0.0,)),
    ((1, 1, 1), lambda q: 2 * (1 - np.cos(q)) + (1 - np.cos(2 * q)),
     lambda q: (np.sin(q) / 3 + np.sin(2 * q) / 3,) * 3),
]


@pytest.mark.parametrize("direction,lam,grad", CASES)
@pytest.mark.parametrize("m", [1, 2, 3])
def test_plane_wave_symbols(direction, lam, grad, m):
    x, y, z = coords(S)
    q = 2 * np.pi * m / S
    ph = q * (direction[0] * x + direction[1] * y + direction[2] * z)
    psi = np.cos(ph)
    assert np.allclose(oracle.laplacian(psi), -lam(q) * psi, atol=1e-13)
    g = oracle.gradient(psi)
    for d in range(3):
        assert np.allclose(g[d], -grad(q)[d] * np.sin(ph), atol=1e-13)


def test_operators_permute_with_axes():
    """Swapping x and y of the field swaps the gradient components."""
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(S ** 3).reshape(S, S, S)
    g = oracle.gradient(psi).reshape(3, S, S, S)
    psiT = np.ascontiguousarray(psi.transpose(0, 2, 1))   # [z, x, y] as [z, y, x]
    gT = oracle.gradient(psiT).reshape(3, S, S, S)
    assert np.allclose(gT[0], g[1].transpose(0, 2, 1), atol=1e-14)
    assert np.allclose(gT[1], g[0].transpose(0, 2, 1), atol=1e-14)
    assert np.allclose(gT[2], g[2].transpose(0, 2, 1), atol=1e-14)


def _free_energy(rho, a, b, kappa, rho_c, S):
    """Discrete Ginzburg-Landau free energy (Sec. II A, Eqs. (fef), (landau-pot))
    with the square-gradient term written over lattice links:
    (3 kappa / 2) sum_r sum_i w_i (rho(r + c_i) - rho(r))^2, which tends to
    kappa/2 |grad rho|^2 in the continuum."""
    r = rho.reshape(S, S, S)
    d = r - rho_c
    F = np.sum(a / 2 * d ** 2 + b / 4 * d ** 4)
    c, w, _, _ = oracle.lattice()
    for i in range(1, 19):
        sh = np.roll(r, shift=(-c[i][2], -c[i][1], -c[i][0]), axis=(0, 1, 2))
        F += 1.5 * kappa * w[i] * np.sum((sh - r) ** 2)
    return F


def test_chemical_potential_is_functional_derivative():
    rng = np.random.default_rng(11)
    S6 = 6
    rho = 1.0 + 0.05 * rng.standard_normal(S6 ** 3)
    a, b, kappa, rho_c = -0.03, 0.7, 0.2, 1.01
    prm = oracle.params(a=a, b=b, kappa=kappa, rho_c=rho_c)
    mu = oracle.chem_potential(rho, prm)
    eps = 1e-5
    for s in rng.choice(S6 ** 3, size=12, replace=False):
        rp, rm = rho.copy(), rho.copy()
        rp[s] += eps
        rm[s] -= eps
        num = (_free_energy(rp, a, b, kappa, rho_c, S6) - _free_energy(rm, a, b, kappa, rho_c, S6)) / (2 * eps)
        assert abs(num - mu[s]) < 1e-8 * max(1.0, abs(mu[s]))


def test_force_plane_wave():
    """b = 0, rho = 1 + eps cos(q x): with the symbols above,
    mu = [a + 2 kappa (1 - cos q)] eps cos(q x) and
    F_x = [rho (a + 2 kappa (1 - cos q)) - 1/3] eps sin q sin(q x)."""
    x, y, z = coords(S)
    a, kappa, eps = 0.05, 0.1, 1e-2
    for m in (1, 3):
        q = 2 * np.pi * m / S
        rho = 1.0 + eps * np.cos(q * x)
        prm = oracle.params(a=a, kappa=kappa, rho_c=1.0)
        mu = oracle.chem_potential(rho, prm)
        assert np.allclose(mu, (a + 2 * kappa * (1 - np.cos(q))) * eps * np.cos(q * x), atol=1e-14)
        F = oracle.force(rho, mu, prm)
        expect = (rho * (a + 2 * kappa * (1 - np.cos(q))) - 1 / 3) * eps * np.sin(q) * np.sin(q * x)
        assert np.allclose(F[0], expect, atol=1e-14)
        assert np.allclose(F[1:], 0, atol=1e-15)
    # force switched off: ideal lattice gas
    off = oracle.params(a=a, kappa=kappa, force_off=True)
    assert np.all(oracle.force(rho, oracle.chem_potential(rho, off), off) == 0)


def test_total_force_vanishes_for_quadratic_free_energy():
    """For b = 0 the force is the action of antisymmetric difference operators
    on the field, so sum_r F = 0 and momentum is conserved exactly; the quartic
    term breaks this (a property of the potential form rho grad mu)."""
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.05 * rng.standard_normal(S ** 3)
    prm = oracle.params(a=0.02, b=0.0, kappa=0.1)
    F = oracle.force(rho, oracle.chem_potential(rho, prm), prm)
    assert np.max(np.abs(F.sum(axis=1))) < 1e-13
    prm_b = oracle.params(a=0.02, b=0.5, kappa=0.1)
    Fb = oracle.force(rho, oracle.chem_potential(rho, prm_b), prm_b)
    assert np.max(np.abs(Fb.sum(axis=1))) > 1e-8
