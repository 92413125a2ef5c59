"""Pins of the oracle's full time step: a dense brute-force implementation on a
small lattice, exact conservation, lattice symmetry and the initial state."""
import numpy as np
import pytest

import oracle

C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
              (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=int)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def idx(S, x, y, z):
    return (x % S) + S * ((y % S) + S * (z % S))


def dense_step(f, S, a, b, kappa, rho_c, tau):
    """Brute force, deterministic part (kT = 0): shift operators as explicit
    N x N permutation matrices, population-space BGK with Guo forcing, and
    streaming by permutation."""
    N = S ** 3
    shift = []
    for i in range(19):               # (Sh_i psi)(r) = psi(r + c_i)
        M = np.zeros((N, N))
        for z in range(S):
            for y in range(S):
                for x in range(S):
                    M[idx(S, x, y, z), idx(S, x + C[i, 0], y + C[i, 1], z + C[i, 2])] = 1
        shift.append(M)
    Lap = 6 * sum(W[i] * (shift[i] - np.eye(N)) for i in range(1, 19))
    Grad = [3 * sum(W[i] * C[i, d] * shift[i] for i in range(1, 19)) for d in range(3)]
    rho = f.sum(axis=0)
    j = C.T.astype(float) @ f
    d = rho - rho_c
    mu = a * d + b * d ** 3 - kappa * (Lap @ rho)
    F = np.array([-rho * (Grad[k] @ mu) + (Grad[k] @ rho) / 3 for k in range(3)])
    u = (j + F / 2) / rho
    cu = C.astype(float) @ u
    cF = C.astype(float) @ F
    u2 = np.sum(u * u, axis=0)
    uF = np.sum(u * F, axis=0)
    feq = W[:, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u2)
    guo = (1 - 1 / (2 * tau)) * W[:, None] * (3 * (cF - uF) + 9 * cu * cF)
    fpost = f - (f - feq) / tau + guo
    out = np.zeros_like(f)
    for i in range(19):               # f_i(r, t+1) = f*_i(r - c_i)
        out[i] = shift[i].T @ fpost[i]
    return out


@pytest.mark.parametrize("tau", [0.7, 1.0, 1.3])
def test_step_matches_dense_brute_force(tau):
    S = 4
    rng = np.random.default_rng(int(tau * 10))
    rho = 1.0 + 0.05 * rng.standard_normal(S ** 3)
    u = 0.02 * rng.standard_normal((3, S ** 3))
    cu = C.astype(float) @ u
    f = W[:, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * np.sum(u * u, axis=0))
    f += 0.003 * W[:, None] * rng.standard_normal(f.shape)
    prm = dict(a=-0.02, b=0.8, kappa=0.12, rho_c=1.01, kT=0.0, tau=tau)
    sim = oracle.Sim(S, seed=1, f=f, nthreads=1, **prm)
    sim.step(1)
    ref = dense_step(f, S, prm["a"], prm["b"], prm["kappa"], prm["rho_c"], tau)
    assert np.max(np.abs(sim.f - ref)) < 1e-15


def test_noise_is_additive_and_conserving():
    """The step with kT > 0 differs from kT = 0 only by the streamed noise,
    which carries no mass or momentum out of any site."""
    S = 5
    base = oracle.Sim(S, seed=77, a=0.01, b=0.3, kappa=0.1, kT=0.0, tau=0.9, init_sigma=0.02, nthreads=1)
    f0 = base.f.copy()
    noisy = oracle.Sim(S, seed=77, a=0.01, b=0.3, kappa=0.1, kT=1e-4, tau=0.9, f=f0, nthreads=1)
    base.step(1)
    noisy.step(1)
    theta = noisy.f - base.f
    # undo streaming: theta_i(r - c_i) was added at site r - c_i
    th = np.zeros_like(theta)
    for i in range(19):
        th[i] = np.roll(theta[i].reshape(S, S, S), shift=(-C[i, 2], -C[i, 1], -C[i, 0]),
                        axis=(0, 1, 2)).reshape(-1)
    assert np.max(np.abs(th.sum(axis=0))) < 1e-15
    assert np.max(np.abs(C.T.astype(float) @ th)) < 1e-15
    assert np.std(th) > 1e-4


def test_mass_exact_and_momentum_budget():
    S = 8
    sim = oracle.Sim(S, seed=2012, a=0.0, b=0.1, kappa=0.1, kT=1e-4, tau=1.0, nthreads=4)
    m0 = sim.f.sum()
    for _ in range(20):
        rho, j = sim.fields()
        mu = oracle.chem_potential(rho, sim.prm)
        F = oracle.force(rho, mu, sim.prm)
        P0 = j.sum(axis=1)
        sim.step(1)
        P1 = sim.fields()[1].sum(axis=1)
        # momentum changes by the total force (R17: exact only for b = 0)
        assert np.allclose(P1 - P0, F.sum(axis=1), atol=1e-13)
    # mass: each step moves the total only by the rounding of the 19-term
    # back-transform sums (a few ulp per site)
    prev = sim.f.sum()
    for _ in range(200):
        sim.step(1)
        cur = sim.f.sum()
        assert abs(cur - prev) / m0 < 19 * np.finfo(float).eps
        prev = cur
    assert abs(prev - m0) / m0 < 220 * 19 * np.finfo(float).eps


def test_momentum_conserved_for_b0():
    S = 8
    sim = oracle.Sim(S, seed=3, a=0.05, b=0.0, kappa=0.1, kT=1e-4, tau=0.8, nthreads=4)
    P0 = sim.fields()[1].sum(axis=1)
    sim.step(200)
    assert np.max(np.abs(sim.fields()[1].sum(axis=1) - P0)) < 1e-12


def test_axis_swap_symmetry_without_noise():
    """At kT = 0 the step commutes with exchanging the x and y axes."""
    S = 6
    rng = np.random.default_rng(21)
    rho = 1 + 0.05 * rng.standard_normal(S ** 3)
    u = 0.02 * rng.standard_normal((3, S ** 3))
    cu = C.astype(float) @ u
    f = W[:, None] * rho * (1 + 3 * cu)
    perm = [next(k for k in range(19) if tuple(C[k]) == (C[i, 1], C[i, 0], C[i, 2])) for i in range(19)]

    def swap(ff):
        g = np.empty_like(ff)
        for i in range(19):
            g[perm[i]] = ff[i].reshape(S, S, S).transpose(0, 2, 1).reshape(-1)
        return g

    kw = dict(a=0.02, b=0.4, kappa=0.1, kT=0.0, tau=0.9, nthreads=1)
    s1 = oracle.Sim(S, seed=1, f=f, **kw)
    s2 = oracle.Sim(S, seed=1, f=swap(f), **kw)
    s1.step(3)
    s2.step(3)
    assert np.max(np.abs(swap(s1.f) - s2.f)) < 1e-15


def test_initial_state():
    S = 16
    sim = oracle.Sim(S, seed=20120221, rho_c=1.0, init_sigma=1e-3)
    rho, j = sim.fields()
    assert np.allclose(sim.f, W[:, None] * rho[None, :], atol=1e-16)
    assert np.max(np.abs(j)) < 1e-16
    d = rho - 1.0
    assert abs(d.mean()) < 4e-3 / np.sqrt(S ** 3)
    assert abs(d.std() / 1e-3 - 1) < 0.05
