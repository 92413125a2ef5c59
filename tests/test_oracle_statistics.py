"""Statistical pins of the oracle: long runs against closed forms and the
linearized theory.  These check the noise amplitudes and the force, which no
algebraic identity fixes."""
import itertools

import numpy as np
import pytest

import linear_theory as lt
import oracle
from oracle import moments
from stats_util import binned_mean, jackknife_binder


def _run(S, n_discard, n_samples, every=1, **kw):
    sim = oracle.Sim(S, **kw)
    sim.step(n_discard)
    rho_k, j_k, rhos = [], [], []
    for _ in range(n_samples):
        sim.step(every)
        rho, j = sim.fields()
        rhos.append(rho)
        rho_k.append(np.abs(np.fft.fftn((rho - rho.mean()).reshape(S, S, S))) ** 2 / S ** 3)
        j_k.append(np.abs(np.fft.fftn(j.reshape(3, S, S, S), axes=(1, 2, 3))) ** 2 / S ** 3)
    return sim, np.array(rho_k), np.array(j_k), np.array(rhos)


def _live_modes(S, **kw):
    mask = np.zeros((S, S, S), bool)
    for iz, iy, ix in itertools.product(range(S), repeat=3):
        if ix == iy == iz == 0:
            continue
        k = 2 * np.pi * np.array([ix, iy, iz]) / S
        mask[iz, iy, ix] = lt.structure_factor(k, **kw) is not None
    return mask


@pytest.mark.parametrize("tau,tb,tg", [(1.0, 0.0, 0.0), (0.8, 0.0, 0.0), (0.8, 1.3, 0.6)])
def test_ideal_gas_equipartition(tau, tb, tg):
    """Force off: S(k) = 3 rho0 kT and <|j(k)|^2>/N = rho0 kT at all live k
    (Eq. (vel-correl) and the ideal-gas compressibility), also with separate
    bulk and ghost relaxation times (each moment's noise matches its own
    rate)."""
    S, kT = 8, 1e-4
    _, rk, jk, _ = _run(S, 100, 3000, seed=5 + int(10 * tau), kT=kT, tau=tau, force_off=True,
                        init_sigma=0.0, nthreads=4, tau_bulk=tb, tau_ghost=tg)
    live = _live_modes(S, tau=tau, kT=kT, force_off=True, tau_bulk=tb, tau_ghost=tg)
    srho = rk[:, live].mean(axis=1)
    sj = jk[:, :, live].mean(axis=2)
    m, e = binned_mean(srho)
    assert abs(m / (3 * kT) - 1) < max(4 * e / (3 * kT), 0.01)
    assert abs(m / (3 * kT) - 1) < 0.03
    for d in range(3):
        mj, ej = binned_mean(sj[:, d])
        assert abs(mj / kT - 1) < max(4 * ej / kT, 0.01)
        assert abs(mj / kT - 1) < 0.03


def test_gaussian_statics_match_linear_theory():
    """b = 0, a > 0: axis S(k) per mode, the block variance <m_L^2> and the
    Binder cumulant (zero for Gaussian statistics) from a long oracle run agree
    with the linearized model within statistical error."""
    S, a, kappa, kT, tau = 12, 0.05, 0.1, 1e-4, 1.0
    sim, _, _, rhos = _run(S, 300, 4000, every=4, seed=99, a=a, b=0.0, kappa=kappa, kT=kT,
                           tau=tau, init_sigma=1e-3, nthreads=8)
    # axis structure factor, averaged over the three axes
    sk = np.array([moments.axis_structure_factor(moments.order_parameter(r), S).mean(axis=0)
                   for r in rhos])
    mean, err = binned_mean(sk)
    theory = lt.axis_structure_factor(S, tau, a=a, kappa=kappa, kT=kT)
    z = (mean - theory) / err
    assert np.all(np.abs(z) < 4.5), (mean / theory, z)
    assert np.all(np.abs(mean / theory - 1) < 0.08)
    # block moments
    for L in (6, 3):
        vals = [moments.block_values(moments.order_parameter(r), S, L)[0] for r in rhos]
        m2 = np.array([np.mean(v ** 2) for v in vals])
        m4 = np.array([np.mean(v ** 4) for v in vals])
        mm2, e2 = binned_mean(m2)
        th = lt.box_variance(S, L, tau, a=a, kappa=kappa, kT=kT)
        assert abs(mm2 - th) < 4.5 * e2 + 0.01 * th, (L, mm2, th, e2)
        U, eU = jackknife_binder(m2, m4)
        assert abs(U) < 4.5 * eU + 0.02, (L, U, eU)
