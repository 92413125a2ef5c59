"""Brute-force pin of the linearized theory on a 4^3 lattice, in real space.

``linear_theory`` predicts the stationary structure factor from 19 x 19
matrices per wave vector, written from the model's definition.  Here the
same prediction is rebuilt from the oracle's own step, with no Fourier
analysis and no noise formula:

- the 1216 x 1216 Jacobian A of one deterministic oracle step (kT = 0)
  around the rest state, by central differences of the oracle itself;
- the noise of one step, f(t+1) - f(t) from the rest state, is linear in
  the step's 15 x 64 normals, which the oracle exposes (site_normals): the
  1216 x 960 map B is recovered by least squares from 1200 oracle steps at
  different step counts, and Q = B B^T;
- the stationary covariance Sigma = sum_n A^n Q A^nT (a discrete Lyapunov
  sum, by doubling; mass, momentum and the frozen zone-edge modes carry no
  noise, so the sum converges).

Its density structure factor must equal linear_theory's at every live mode
(two independent constructions of the same linear statistics), and long
oracle runs must match it within their statistical error (the nonlinear
terms are negligible at this noise level).
"""
import numpy as np
import pytest

import linear_theory as lt
import oracle
from stats_util import binned_mean

S = 4
N = S ** 3
Q = 19
PRM = dict(a=0.05, b=0.0, kappa=0.1, rho_c=1.0, tau=0.9)
KT = 1e-4


def _step(f, kT, t=0, seed=7):
    sim = oracle.Sim(S, seed, f=f, t=t, kT=kT, nthreads=1, **PRM)
    sim.step(1)
    return sim.f


@pytest.fixture(scope="module")
def linear_model():
    _, w, _, _ = oracle.lattice()
    f0 = np.repeat(w[:, None] * PRM["rho_c"], N, axis=1)
    assert np.allclose(_step(f0, 0.0), f0, rtol=0, atol=1e-15)  # the rest state is a fixed point
    n = Q * N
    h = 1e-6
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        A[:, k] = (_step(f0 + e.reshape(Q, N), 0.0) - _step(f0 - e.reshape(Q, N), 0.0)).reshape(-1) / (2 * h)
    # noise map: f(t+1) - f0 = B g(t), g the 15 normals of each of the 64 sites at step t
    seed, steps = 11, 1200
    X = np.zeros((steps, n))
    G = np.zeros((steps, 15 * N))
    for t in range(steps):
        X[t] = (_step(f0, KT, t=t, seed=seed) - f0).reshape(-1)
        G[t] = np.concatenate([oracle.site_normals(seed, s, t, 0)[:15] for s in range(N)])
    B, res, rank, _ = np.linalg.lstsq(G, X, rcond=None)
    assert rank == 15 * N
    assert np.max(np.abs(G @ B - X)) < 1e-12 * np.max(np.abs(X))  # exactly linear in the normals
    Qn = B.T @ B
    # Sigma = sum_{n < 2^16} A^n Q A^nT by doubling (Sigma_2m = Sigma_m + A^m
    # Sigma_m A^mT): every noised mode relaxes within a few hundred steps,
    # while the modes that do not relax (mass, k = 0 momentum, the frozen
    # zone-edge ones) receive no noise and drop out of the comparison
    Psum = np.kron(np.ones((1, Q)), np.eye(N))          # rho(x) = sum_i f_i(x)

    def density_sk(Sig):
        # C(k) = N^-1 sum_{x,y} e^{-ik.(x - y)} Cov(rho_x, rho_y): the diagonal of
        # the transform over x (e^{-ik.x}) and the inverse transform over y (its 1/N)
        C6 = (Psum @ Sig @ Psum.T).reshape(S, S, S, S, S, S)
        M = np.fft.ifftn(np.fft.fftn(C6, axes=(0, 1, 2)), axes=(3, 4, 5))
        idx = np.arange(S)
        return np.real(M[idx[:, None, None], idx[None, :, None], idx[None, None, :],
                         idx[:, None, None], idx[None, :, None], idx[None, None, :]])

    Sig, P = Qn.copy(), A.copy()
    prev = None
    for _ in range(16):
        Sig = Sig + P @ Sig @ P.T
        P = P @ P
        cur = density_sk(Sig)
        if prev is not None:
            live = [m for m, _ in _modes()]
            if max(abs(cur[m] / prev[m] - 1) for m in live) < 1e-13:
                break
        prev = cur
    else:
        raise AssertionError("Lyapunov sum did not converge on the live modes")
    return cur


def _modes():
    out = []
    for iz in range(S):
        for iy in range(S):
            for ix in range(S):
                if ix == iy == iz == 0:
                    continue
                k = 2 * np.pi * np.array([ix, iy, iz]) / S
                v = lt.structure_factor(k, PRM["tau"], a=PRM["a"], kappa=PRM["kappa"], kT=KT, rho0=PRM["rho_c"])
                if v is not None:
                    out.append(((iz, iy, ix), v))
    return out


def test_real_space_lyapunov_equals_per_k_theory(linear_model):
    modes = _modes()
    assert len(modes) >= 40
    worst = 0.0
    for (iz, iy, ix), th in modes:
        got = linear_model[iz, iy, ix]
        worst = max(worst, abs(got / th - 1))
        assert abs(got / th - 1) < 1e-8, ((ix, iy, iz), got, th)   # central differences of step h = 1e-6
    print(f"{len(modes)} live modes, worst relative difference {worst:.1e}")


def test_long_oracle_run_matches_real_space_theory(linear_model):
    """4^3, a = 0.05, b = 0, kT = 1e-4: 60000 sampled steps of the oracle,
    per-mode S(k) within five standard errors of the real-space prediction."""
    sim = oracle.Sim(S, 23, kT=KT, nthreads=1, init_sigma=0.0, **PRM)
    sim.step(500)
    acc = []
    for _ in range(60000):
        sim.step(1)
        rho = sim.fields()[0].reshape(S, S, S)
        acc.append(np.abs(np.fft.fftn(rho - rho.mean())) ** 2 / N)
    acc = np.array(acc)
    mean, err = binned_mean(acc, nbins=30)
    zs = []
    for (iz, iy, ix), _ in _modes():
        th = linear_model[iz, iy, ix]
        zs.append((mean[iz, iy, ix] - th) / err[iz, iy, ix])
    zs = np.array(zs)
    print(f"max |z| {np.max(np.abs(zs)):.2f}")
    assert np.all(np.abs(zs) < 5), zs
    # and on average over the live modes within 2%
    ratio = np.mean([mean[m] / linear_model[m] for m, _ in _modes()])
    print(f"mean S_oracle / S_linear {ratio:.4f}")
    assert abs(ratio - 1) < 0.02, ratio
