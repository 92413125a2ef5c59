"""Pins of the oracle's moment-space collision.

With all non-conserved moments relaxed at the same rate, the moment-space
collision must coincide with the textbook population-space BGK collision of
Eq. (lbe) with the second-order equilibrium
  f_i^eq = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2]
and Guo's forcing term (Guo, Zheng, Shi 2002)
  (1 - 1/(2 tau)) w_i [3 (c - u) . F + 9 (c . u)(c . F)],  u = (j + F/2)/rho.
The noise must leave density and momentum untouched (Eq. (lbnoise): rows and
columns of the conserved moments vanish)."""
import numpy as np
import pytest

import oracle

C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
              (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def textbook_bgk_guo(f, F, tau):
    rho = f.sum()
    j = C.T @ f
    u = (j + F / 2) / rho
    cu = C @ u
    feq = W * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
    guo = (1 - 1 / (2 * tau)) * W * (3 * ((C - u) @ F) + 9 * cu * (C @ F))
    return f - (f - feq) / tau + guo


@pytest.mark.parametrize("tau", [0.51, 0.8, 1.0, 1.7, 5.0])
def test_collision_equals_textbook_bgk_guo(tau):
    rng = np.random.default_rng(int(tau * 100))
    # C order matches the oracle's table (checked in the lattice tests)
    c, _, _, _ = oracle.lattice()
    assert np.array_equal(c, C.astype(int))
    for _ in range(20):
        rho = 1 + 0.2 * rng.standard_normal()
        u = 0.05 * rng.standard_normal(3)
        cu = C @ u
        f = W * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u) + 0.01 * rng.standard_normal(19) * W
        F = 0.01 * rng.standard_normal(3)
        prm = oracle.params(a=0.3, b=0.2, kappa=0.1, kT=0.0, tau=tau)
        got = oracle.collide_site(prm, f, F)
        assert np.allclose(got, textbook_bgk_guo(f, F, tau), atol=1e-14, rtol=0)


def test_collision_conserves_mass_and_adds_force():
    rng = np.random.default_rng(7)
    f = W * (1 + 0.1 * rng.standard_normal(19))
    F = 0.02 * rng.standard_normal(3)
    g = rng.standard_normal(16)
    prm = oracle.params(kT=1e-3, tau=0.9)
    out = oracle.collide_site(prm, f, F, g)
    assert abs(out.sum() - f.sum()) < 1e-15
    assert np.allclose(C.T @ out, C.T @ f + F, atol=1e-15)


def test_noise_projection_and_amplitude():
    """theta = collide(g) - collide(0) has zero mass and momentum; its moment a
    (a >= 4) is sigma_a g_{a-4}, sigma_a^2 = rho kT (1/tau)(2 - 1/tau) N_a / c_s^2."""
    rng = np.random.default_rng(9)
    f = W * (1.1 + 0.05 * rng.standard_normal(19))
    F = np.zeros(3)
    g = rng.standard_normal(16)
    tau, kT = 0.8, 2e-4
    prm = oracle.params(kT=kT, tau=tau)
    theta = oracle.collide_site(prm, f, F, g) - oracle.collide_site(prm, f, F, np.zeros(16))
    assert abs(theta.sum()) < 1e-16 and np.max(np.abs(C.T @ theta)) < 1e-16
    _, _, T, n = oracle.lattice()
    rho = f.sum()
    sig = np.sqrt(rho * kT * (1 / tau) * (2 - 1 / tau) * n[4:] * 3)
    assert np.allclose(T[4:] @ theta, sig * g[:15], atol=1e-15)


def test_unstable_density_is_reported():
    f = -W * 0.1
    with pytest.raises(FloatingPointError):
        oracle.collide_site(oracle.params(tau=1.0), f, np.zeros(3))


def test_separate_rates_touch_only_their_moments():
    """Separate relaxation times (bulk: moment 4, ghosts: 10..18; the paper
    sets every time to one value, Sec. III B): without noise and force, the
    ghost time changes none of the moments 0..9 after collision, the bulk
    time only moment 4, and equal times reproduce the BGK collision exactly."""
    rng = np.random.default_rng(12)
    _, _, T, n = oracle.lattice()
    f = W * (1.05 + 0.05 * rng.standard_normal(19))
    F = np.zeros(3)
    base = oracle.collide_site(oracle.params(tau=0.8), f, F)
    same = oracle.collide_site(oracle.params(tau=0.8, tau_bulk=0.8, tau_ghost=0.8), f, F)
    assert np.array_equal(base, same)
    ghost = oracle.collide_site(oracle.params(tau=0.8, tau_ghost=1.7), f, F)
    assert np.allclose(T[:10] @ ghost, T[:10] @ base, atol=1e-15)
    assert np.max(np.abs(T[10:] @ (ghost - base))) > 1e-4
    bulk = oracle.collide_site(oracle.params(tau=0.8, tau_bulk=1.9), f, F)
    d = T @ (bulk - base)
    assert abs(d[4]) > 1e-5 and np.max(np.abs(np.delete(d, 4))) < 1e-15


def test_noise_amplitude_with_separate_rates():
    """Moment a gets sigma_a^2 = rho kT (1 - gamma_a^2) N_a / c_s^2 with its own gamma_a."""
    rng = np.random.default_rng(13)
    f = W * (1.1 + 0.05 * rng.standard_normal(19))
    g = rng.standard_normal(16)
    tau, tb, tg, kT = 0.8, 1.4, 0.6, 2e-4
    prm = oracle.params(kT=kT, tau=tau, tau_bulk=tb, tau_ghost=tg)
    theta = oracle.collide_site(prm, f, np.zeros(3), g) - oracle.collide_site(prm, f, np.zeros(3), np.zeros(16))
    _, _, T, n = oracle.lattice()
    taus = np.array([tb] + [tau] * 5 + [tg] * 9)
    gam = 1 - 1 / taus
    sig = np.sqrt(f.sum() * kT * (1 - gam ** 2) * n[4:] * 3)
    assert np.allclose(T[4:] @ theta, sig * g[:15], atol=1e-15)
