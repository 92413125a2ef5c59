"""Long GPU runs against what the model fixes statistically.

- Gaussian statics (b = 0, a > 0) at 64^3: the axis structure factor per
  mode and the block variances against the linearized model (19x19 discrete
  Lyapunov per wave vector), whose small-k limit is the Ornstein-Zernike form
  kT / (a + kappa_eff k^2) of Sec. II A, Eq. (CMF); Binder cumulant zero.
- Ideal lattice gas (force off): S(k) = 3 kT at every axis mode.
- b > 0 (no closed form): GPU statistics against oracle statistics on a small
  lattice (the same seeded trajectory and an independent seed).
- FP16 storage against FP32 storage on the same seed (precision variant).

Errors are batch-means errors from independent windows of the run.
"""
import numpy as np
import pytest

import linear_theory as lt
import oracle
import workloads
from oracle import moments
from gpu_util import require_gpu, say
from stats_util import binned_mean, jackknife_binder

pytestmark = pytest.mark.gpu


def _windows(sim, n_windows, steps_per_window, L):
    """Axis S(k) (averaged over the three axes) and level moments per window."""
    sks, levs = [], []
    for _ in range(n_windows):
        sim.reset_moments()
        sim.step(steps_per_window)
        m = sim.moments()
        sks.append(m["sk"].mean(axis=0) / m["n_samples"])
        levs.append({lv["Lb"]: (lv["m2"] / (lv["n_boxes"] * m["n_samples"]),
                                lv["m4"] / (lv["n_boxes"] * m["n_samples"])) for lv in m["levels"]})
    return np.array(sks), levs


def test_gaussian_statics_64():
    """64^3, b = 0, a = 0.05, kappa = 0.1, kT = 1e-4, tau = 1 (the verification
    run of the 64^3 workload): 3500 steps discarded, 16500 sampled every 10."""
    lbf = require_gpu()
    L = 64
    prm = dict(workloads.WORKLOADS["d3q19_64_oz"])
    prm.pop("L"), prm.pop("steps")
    say("statics 64^3 b=0")
    sim = lbf.Sim(L, workloads.SEED + 1, sample_every=10, series_capacity=2048, **prm)
    sim.step(3500)
    sks, levs = _windows(sim, 15, 1100, L)
    mean, err = binned_mean(sks, nbins=15)
    theory = lt.axis_structure_factor(L, prm["tau"], a=prm["a"], kappa=prm["kappa"], kT=prm["kT"])
    z = (mean - theory) / err
    say(f"  S/S_lin (m=1..8): {np.round(mean[:8] / theory[:8], 4)}")
    say(f"  max |z| {np.max(np.abs(z)):.2f}")
    assert np.all(np.abs(z) < 5), z
    # small k: the Ornstein-Zernike form with the lattice-shifted kappa
    for mi in (1, 2):
        k = 2 * np.pi * mi / L
        oz = prm["kT"] / (prm["a"] + (prm["kappa"] + 1 / 12) * k * k)
        assert abs(mean[mi - 1] / oz - 1) < 5 * err[mi - 1] / oz + 0.02
    # block variances and Binder cumulant of Gaussian statistics
    for Lb in (16, 8, 4):
        m2 = np.array([lv[Lb][0] for lv in levs])
        m4 = np.array([lv[Lb][1] for lv in levs])
        mm2, e2 = binned_mean(m2, nbins=15)
        th = lt.box_variance(L, Lb, prm["tau"], a=prm["a"], kappa=prm["kappa"], kT=prm["kT"])
        say(f"  L_b={Lb}: <m^2> {mm2:.4e} +- {e2:.1e}, linear theory {th:.4e}")
        assert abs(mm2 - th) < 5 * e2 + 0.02 * th
        U, eU = jackknife_binder(m2, m4, nbins=15)
        assert abs(U) < 5 * eU + 0.01, (Lb, U, eU)


@pytest.mark.parametrize("rates", [{}, {"tau_bulk": 1.3, "tau_ghost": 0.6}])
def test_ideal_gas_structure_factor_32(rates):
    """Force off: S(k) = 3 kT at every axis mode, with one relaxation time and
    with separate bulk and ghost times (fluctuation-dissipation per moment)."""
    lbf = require_gpu()
    L, kT = 32, 1e-4
    say(f"ideal gas 32^3 {rates}")
    sim = lbf.Sim(L, 5, kT=kT, tau=0.8, force_off=True, init_sigma=0.0, sample_every=5, **rates)
    sim.step(500)
    sks, _ = _windows(sim, 12, 1000, L)
    mean, err = binned_mean(sks, nbins=12)
    live = mean[:-1]  # every axis mode below the zone edge
    assert np.all(np.abs(live / (3 * kT) - 1) < 5 * err[:-1] / (3 * kT) + 0.01)
    assert abs(np.mean(live) / (3 * kT) - 1) < 0.01


def test_quartic_statistics_against_oracle():
    """a = 0, b = 0.1 at 12^3 (no closed form): block <m^2>, <m^4>, Binder and
    S(k) from the GPU agree with the oracle's on the same seed within the
    statistical error of an independent seed."""
    lbf = require_gpu()
    L, steps, every = 12, 12000, 4
    prm = dict(workloads.MODEL)
    say("quartic 12^3 gpu vs oracle")
    res = {}
    for who, seed in (("gpu", 31), ("oracle", 31), ("gpu2", 32)):
        if who.startswith("gpu"):
            sim = lbf.Sim(L, seed, sample_every=every, series_capacity=steps // every, **prm)
            sim.step(steps)
            ser = sim.moments(series=True)["series"]
            m2 = ser[:, 5 + 7 * 0 + 1]   # level L_b = 6: box mean of m^2
            m4 = ser[:, 5 + 7 * 0 + 3]
        else:
            orc = oracle.Sim(L, seed, **prm)
            m2, m4 = [], []
            for _ in range(steps // every):
                orc.step(every)
                mm, _E = moments.block_values(moments.order_parameter(orc.rho()), L, 6)
                m2.append(np.mean(mm ** 2))
                m4.append(np.mean(mm ** 4))
            m2, m4 = np.array(m2), np.array(m4)
        burn = len(m2) // 6
        res[who] = (m2[burn:], m4[burn:])
    g2, g4 = res["gpu"]
    o2, o4 = res["oracle"]
    # same seed: the FP32 and FP64 trajectories stay together sample by sample
    assert np.max(np.abs(g2 - o2)) < 1e-3 * np.max(np.abs(o2))
    mg, eg = binned_mean(res["gpu2"][0], nbins=10)
    mo, eo = binned_mean(o2, nbins=10)
    assert abs(mg - mo) < 5 * np.hypot(eg, eo)
    Ug, eUg = jackknife_binder(*res["gpu2"], nbins=10)
    Uo, eUo = jackknife_binder(o2, o4, nbins=10)
    say(f"  Binder L_b=6: gpu {Ug:.4f} +- {eUg:.4f}, oracle {Uo:.4f} +- {eUo:.4f}")
    assert abs(Ug - Uo) < 5 * np.hypot(eUg, eUo)


def test_fp16_precision_variant():
    """FP16 deviation storage against FP32 storage, same seed: mass drift and
    the structure factor at the resolved modes (b = 0, a = 0.05, 96^3)."""
    lbf = require_gpu()
    L = 96
    prm = dict(workloads.MODEL, a=0.05, b=0.0)
    say("fp16 vs fp32 96^3")
    out = {}
    for storage in ("fp32", "fp16"):
        sim = lbf.Sim(L, 77, storage=storage, sample_every=10, **prm)
        m0 = sim.moments()["mass"]
        sim.step(1000)
        sim.reset_moments()
        sim.step(4000)
        m = sim.moments()
        out[storage] = (m["sk"].mean(axis=0) / m["n_samples"], abs(m["mass"] - m0) / m0)
    sk32, drift32 = out["fp32"]
    sk16, drift16 = out["fp16"]
    say(f"  mass drift fp32 {drift32:.2e}, fp16 {drift16:.2e}")
    assert drift32 < 1e-7 and drift16 < 1e-5
    theory = lt.axis_structure_factor(L, prm["tau"], a=prm["a"], kappa=prm["kappa"], kT=prm["kT"])
    sel = slice(8, L // 2 - 1)   # modes that relax within the run
    r16 = sk16[sel] / theory[sel]
    r32 = sk32[sel] / theory[sel]
    say(f"  S16/S_lin mean {r16.mean():.4f}, S32/S_lin mean {r32.mean():.4f}")
    assert abs(r16.mean() - 1) < 0.03 and abs(r32.mean() - 1) < 0.03
    assert abs(r16.mean() - r32.mean()) < 0.02
