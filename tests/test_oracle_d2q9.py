"""Pins of the oracle of the paper's own D2Q9 model (Sec. III A): the
equilibrium against the paper's explicit population formula and Eq.
(holdych-cond), the noise factor against Eq. (lbnoise), the random numbers
against the D3Q19 oracle's generator, exact conservation, lattice symmetry
and the equilibrium statistics (S(k) = kT/(a + kappa k^2), Eq. (CMF);
<|j(k)|^2> = rho0 kT, Eq. (vel-correl))."""
import os

import numpy as np
import pytest

import oracle
from oracle import d2q9 as D

PRM = dict(a=0.05, b=0.7, kappa=0.02, rho_c=1.0, kT=1e-5, tau=0.8)


def _state(L, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * rng.standard_normal(L * L)
    j = 0.02 * rng.standard_normal((2, L * L))
    return rho, j


def _paper_feq(rho, j, L, prm):
    """The equilibrium written population by population as the paper prints
    it (Sec. III A), with three misprints read as: kappa in front of
    rho lap rho, (d_x rho)^2 for the w^xx term, and a plus sign before the
    u.grad rho delta term."""
    a, b, kappa, rho_c, tau = prm["a"], prm["b"], prm["kappa"], prm["rho_c"], prm["tau"]
    d = rho - rho_c
    p0 = rho * (a * d + b * d ** 3) - (0.5 * a * d * d + 0.25 * b * d ** 4)
    gx, gy = D.gradient(rho, L)
    lap = D.laplacian(rho, L)
    ux, uy = j / rho
    nu = (tau - 0.5) / 3
    A = {(0, 0): rho * ux * ux + nu * (2 * ux * gx + ux * gx + uy * gy),
         (1, 1): rho * uy * uy + nu * (2 * uy * gy + ux * gx + uy * gy),
         (0, 1): rho * ux * uy + nu * (ux * gy + uy * gx)}
    A[(1, 0)] = A[(0, 1)]
    w = [None, 1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12]
    wxx = [None, 1 / 3, 1 / 3, -1 / 6, -1 / 6, -1 / 24, -1 / 24, -1 / 24, -1 / 24]
    wyy = [None, -1 / 6, -1 / 6, 1 / 3, 1 / 3, -1 / 24, -1 / 24, -1 / 24, -1 / 24]
    wxy = [None, 0, 0, 0, 0, 1 / 4, 1 / 4, -1 / 4, -1 / 4]
    f = np.zeros((9, rho.size))
    for i in range(1, 9):
        c = D.C[i]
        tens = sum(1.5 * (c[p] * c[q] - (1 / 3) * (p == q)) * A[(p, q)] for p in range(2) for q in range(2))
        f[i] = (w[i] * (rho * (ux * c[0] + uy * c[1]) + tens + p0 - kappa * rho * lap)
                + wxx[i] * kappa * gx * gx + wyy[i] * kappa * gy * gy + wxy[i] * kappa * gx * gy)
    f[0] = rho - f[1:].sum(axis=0)
    return f


def test_equilibrium_is_the_papers_formula():
    L = 6
    rho, j = _state(L, 1)
    got = D.equilibrium(rho, j, L, PRM)
    ref = _paper_feq(rho, j, L, PRM)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_equilibrium_moments_satisfy_the_pressure_condition():
    """Eq. (holdych-cond) with the pressure tensor of Eq. (press-th)."""
    L = 6
    rho, j = _state(L, 2)
    f = D.equilibrium(rho, j, L, PRM)
    c = D.C.astype(float)
    assert np.allclose(f.sum(axis=0), rho, atol=1e-15, rtol=0)
    assert np.allclose(c.T @ f, j, atol=1e-15, rtol=0)
    k, tau = PRM["kappa"], PRM["tau"]
    d = rho - 1.0
    p0 = rho * (PRM["a"] * d + PRM["b"] * d ** 3) - (PRM["a"] * d * d / 2 + PRM["b"] * d ** 4 / 4)
    g = D.gradient(rho, L)
    lap = D.laplacian(rho, L)
    u = j / rho
    nu = (tau - 0.5) / 3
    for p in range(2):
        for q in range(2):
            Pi = (c[:, p] * c[:, q]) @ f
            P = (p0 - k * rho * lap - k / 2 * (g ** 2).sum(axis=0)) * (p == q) + k * g[p] * g[q]
            want = P + rho * u[p] * u[q] + nu * (u[p] * g[q] + u[q] * g[p] + (u * g).sum(axis=0) * (p == q))
            assert np.allclose(Pi, want, atol=1e-15, rtol=0)


def test_noise_factor_against_the_printed_matrix():
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_lbnoise_d2q9_matrix.txt")
    with open(path) as fh:
        ent = [tuple(float(v) for v in line.split()) for line in fh if line.strip() and not line.startswith("#")]
    for x in (-0.3, 0.0, 0.01, 1 / 3, 0.5, 0.59):
        M = np.zeros((6, 6))
        for r, cc, c0, c1 in ent:
            M[int(r) - 3, int(cc) - 3] = M[int(cc) - 3, int(r) - 3] = c0 + c1 * x
        L33, L83, L88, dg = D.noise_factor(np.array([x]))
        Lm = np.zeros((6, 6))
        Lm[0, 0], Lm[5, 0], Lm[5, 5] = L33[0], L83[0], L88[0]
        for k_ in range(4):
            Lm[1 + k_, 1 + k_] = dg[k_]
        assert np.allclose(Lm @ Lm.T, M, atol=1e-13)
    # at the lattice sound speed the matrix is the basis norms (diagonal)
    L33, L83, L88, dg = D.noise_factor(np.array([1 / 3]))
    assert abs(L83[0]) < 1e-15
    assert np.allclose([L33[0] ** 2, *(dg ** 2), L88[0] ** 2], D.NORM[3:], atol=1e-14)


def test_random_numbers_are_the_d3q19_oracles():
    rng = np.random.default_rng(9)
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        got = [int(v[0]) for v in D.philox(*[np.array([c], dtype=np.uint64) for c in ctr], *key)]
        assert got == oracle.philox(ctr, key)
    g = D.normals(20120221, np.arange(7), 123456789012)
    for s in range(7):
        assert np.array_equal(g[:, s], oracle.site_normals(20120221, s, 123456789012)[:8])


def test_mass_and_momentum_conserved_exactly():
    """No body force: every step conserves sum rho and sum j to rounding,
    for any b and kappa (unlike the force scheme of the D3Q19 model)."""
    sim = D.Sim(12, 4, **dict(PRM, b=2.0, init_sigma=0.02))
    r0, j0 = sim.fields()
    sim.step(40)
    r1, j1 = sim.fields()
    assert abs(r1.sum() - r0.sum()) < 1e-11
    assert np.max(np.abs(j1.sum(axis=1) - j0.sum(axis=1))) < 1e-11


def test_quarter_turn_symmetry():
    """Rotating the state by 90 degrees commutes with a noiseless step."""
    L = 8
    prm = dict(PRM, kT=0.0)
    rng = np.random.default_rng(6)
    f = D.equilibrium(1.0 + 0.03 * rng.standard_normal(L * L), 0.01 * rng.standard_normal((2, L * L)), L, prm)
    f += 1e-3 * rng.standard_normal(f.shape)
    # (x, y) -> (-y, x): velocity i maps to the velocity (-c_y, c_x)
    perm = [next(k for k in range(9) if tuple(D.C[k]) == (-D.C[i][1], D.C[i][0])) for i in range(9)]

    def rot(g):
        out = np.empty_like(g)
        for i in range(9):
            grid = g[i].reshape(L, L)  # [y, x]
            out[perm[i]] = np.rot90(grid, k=1, axes=(1, 0)).reshape(-1)
        return out

    a = D.step(rot(f), L, prm, 1, 0)
    b = rot(D.step(f, L, prm, 1, 0))
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.slow
def test_equilibrium_statistics_16():
    """Eq. (CMF) with the lattice k^2 and Eq. (vel-correl) on a 16^2 lattice:
    S(k) = kT / (a + kappa k^2) and <|j_a(k)|^2>/N = rho0 kT averaged over all
    k != 0 within 4% (b = 0, kappa = 1e-3, tau = 0.8, 8000 sampled steps)."""
    L = 16
    prm = dict(a=0.05, b=0.0, kappa=1e-3, rho_c=1.0, kT=1e-5, tau=0.8, init_sigma=0.0)
    sim = D.Sim(L, 7, **prm)
    sim.step(1500)
    S = np.zeros((L, L))
    J = np.zeros((2, L, L))
    n = 0
    for _ in range(400):
        sim.step(20)
        rho, j = sim.fields()
        S += np.abs(np.fft.fft2(rho.reshape(L, L))) ** 2 / L ** 2
        for a_ in range(2):
            J[a_] += np.abs(np.fft.fft2(j[a_].reshape(L, L))) ** 2 / L ** 2
        n += 1
    m = np.fft.fftfreq(L) * L
    ky, kx = np.meshgrid(2 * np.pi * m / L, 2 * np.pi * m / L, indexing="ij")
    lap = 6 * ((1 / 9) * (2 - 2 * np.cos(kx) + 2 - 2 * np.cos(ky))
               + (1 / 36) * (4 - 2 * np.cos(kx + ky) - 2 * np.cos(kx - ky)))
    th = prm["kT"] / (prm["a"] + prm["kappa"] * lap)
    ratio = (S / n / th).reshape(-1)[1:]
    assert abs(ratio.mean() - 1) < 0.04
    for a_ in range(2):
        assert abs((J[a_] / n).reshape(-1)[1:].mean() / prm["kT"] - 1) < 0.04
