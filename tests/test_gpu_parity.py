"""GPU path against the FP64 oracle, element by element, through the C ABI.

Tolerances (FP32 compute and storage against FP64), after every step:
- max |X_gpu - X_oracle| / max |X_oracle| <= 1e-5 for X in {rho, j, f} (the
  field bound of the target, as a fraction of the largest value);
- || X_gpu - X_oracle ||_2 / || X_oracle - X_rest ||_2 <= DTOL32 for the
  deviations drho (X_rest the mean density) and f - w_i rho_c: the bound held
  to the fluctuation itself, which is ~1e-3 of rho.  Measured worst 2.9e-7
  (16^3, 1000 steps); DTOL32 = 2e-6 keeps a margin of about 7.

FP16 storage rounds each stored deviation r_i = (f_i - w_i rho_c)/w_i
(|r| <~ 0.1) to 11 significant bits, so the FP16 bounds are set by those
roundings: measured worst over 100 steps (16^3) rho 2.0e-5, j 3.4e-4, f
4.3e-5 of the largest value, deviation-relative drho 2.9e-4 and f 2.5e-4;
each bound below is about 5 times the measured worst.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev_rel_err, rel_err, require_gpu, say

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = {"rho": 1e-4, "j": 1.5e-3, "f": 2e-4}
DTOL32 = 2e-6
DTOL16 = 1.5e-3
M0 = workloads.MODEL


def dev_errors(fg, orc):
    """Deviation-relative errors of drho and of f - w rho_c."""
    rho_o, _ = orc.fields()
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)[:, None]
    rest = w * orc.prm.rho_c
    ef = float(np.linalg.norm(fg["f"] - orc.f) / max(np.linalg.norm(orc.f - rest), 1e-300))
    return dev_rel_err(fg["rho"], rho_o), ef


def _compare(sim, orc, tol, where, replica=0, dtol=None):
    fg = sim.fields(replica, rho=True, j=True, f=True)
    rho_o, j_o = orc.fields()
    e = (rel_err(fg["rho"], rho_o), rel_err(fg["j"], j_o), rel_err(fg["f"], orc.f))
    if isinstance(tol, dict):
        ok = e[0] <= tol["rho"] and e[1] <= tol["j"] and e[2] <= tol["f"]
    else:
        ok = max(e) <= tol
    assert ok, f"{where}: rel errors rho/j/f = {e}"
    if dtol is not None:
        d = dev_errors(fg, orc)
        assert max(d) <= dtol, f"{where}: deviation-relative errors drho/f = {d}"
        e = e + d
    return e


def test_initial_state():
    lbf = require_gpu()
    say("initial state L=16")
    sim = lbf.Sim(16, workloads.SEED, **M0)
    orc = oracle.Sim(16, workloads.SEED, **M0)
    _compare(sim, orc, 1e-7, "t=0")


@pytest.mark.parametrize("kernel", ["split", "fused", "rows"])
def test_config0_100_steps(kernel):
    """16^3, a=0, b=0.1, kappa=0.1, kT=1e-4, tau=1: every step of 100."""
    lbf = require_gpu()
    say(f"config0 L=16 kernel={kernel}")
    sim = lbf.Sim(16, workloads.SEED, **M0)
    sim.set_plan(kernel, (16, 16, 8))
    orc = oracle.Sim(16, workloads.SEED, **M0)
    worst = np.zeros(5)
    for t in range(100):
        sim.step(1)
        orc.step(1)
        worst = np.maximum(worst, _compare(sim, orc, TOL32, f"step {t + 1}", dtol=DTOL32))
    say(f"  worst rho/j/f {worst[0]:.2e} {worst[1]:.2e} {worst[2]:.2e}, "
        f"deviation-relative drho/f {worst[3]:.2e} {worst[4]:.2e}")


def test_config0_1000_steps():
    """The whole 16^3 run of 1000 steps on the default plan with graph replay
    and sampling every step, checked at steps 1, 10, 100 and 1000."""
    lbf = require_gpu()
    say("config0 L=16 1000 steps")
    sim = lbf.Sim(16, workloads.SEED, sample_every=1, **M0)
    orc = oracle.Sim(16, workloads.SEED, **M0)
    done = 0
    for t in (1, 10, 100, 1000):
        if t - done >= 8:
            sim.set_plan("rows", (32, 8, 16), graph_steps=8)
        sim.step(t - done)
        orc.step(t - done)
        done = t
        e = _compare(sim, orc, TOL32, f"step {t}", dtol=DTOL32)
        say(f"  step {t}: rho/j/f {e[0]:.2e} {e[1]:.2e} {e[2]:.2e}, drho/f {e[3]:.2e} {e[4]:.2e}")
    assert sim.moments()["n_samples"] == 1000


@pytest.mark.parametrize("L,kernel,tile", [(4, "rows", (16, 16, 4)), (7, "staged", (32, 8, 3)),
                                           (12, "rows", (16, 16, 5)), (12, "staged", (16, 8, 5)),
                                           (20, "rows", (16, 16, 16)), (37, "staged", (32, 8, 16)),
                                           (40, "rows", (32, 8, 7)), (44, "rows", (16, 8, 9)),
                                           (36, "fused", (64, 4, 5)), (36, "rows", (64, 4, 5)),
                                           (40, "rows", (64, 8, 6))])
def test_ragged_sizes(L, kernel, tile):
    """Sizes not divisible by the tile (partial tiles, wrap-around halos, the
    source rows of the rows staging wrapping more than once on L = 4)."""
    lbf = require_gpu()
    say(f"ragged L={L} {kernel} tile={tile}")
    prm = dict(M0, a=0.01, b=0.5, tau=0.8)
    sim = lbf.Sim(L, 7 + L, **prm)
    sim.set_plan(kernel, tile)
    orc = oracle.Sim(L, 7 + L, **prm)
    for t in range(10):
        sim.step(1)
        orc.step(1)
        _compare(sim, orc, TOL32, f"L={L} step {t + 1}", dtol=DTOL32)


def test_strong_nonequilibrium_state():
    """A far-from-equilibrium state (drho 0.05, u 0.03, random ghosts) through
    the import path, with a strong quartic term."""
    lbf = require_gpu()
    L = 12
    say("strong state L=12")
    f0 = workloads.random_populations(L, 99, drho=0.05, u=0.03, neq=0.02)
    prm = dict(a=-0.05, b=2.0, kappa=0.2, rho_c=1.0, kT=1e-4, tau=0.7)
    for kernel in ("split", "fused", "rows"):
        sim = lbf.Sim(L, 5, **prm)
        sim.set_plan(kernel, (16, 16, 4))
        sim.set_populations(f0)
        orc = oracle.Sim(L, 5, f=f0, **prm)
        _compare(sim, orc, 1e-6, f"{kernel} import")
        for t in range(20):
            sim.step(1)
            orc.step(1)
            _compare(sim, orc, TOL32, f"{kernel} step {t + 1}", dtol=DTOL32)


def test_force_off_ideal_gas():
    lbf = require_gpu()
    say("force off L=12")
    prm = dict(M0, force_off=True, tau=0.9)
    sim = lbf.Sim(12, 3, **prm)
    orc = oracle.Sim(12, 3, **prm)
    sim.step(20)
    orc.step(20)
    _compare(sim, orc, TOL32, "force off", dtol=DTOL32)


@pytest.mark.parametrize("kernel", ["split", "rows"])
def test_fp16_storage(kernel):
    lbf = require_gpu()
    say(f"fp16 L=16 {kernel}")
    sim = lbf.Sim(16, workloads.SEED, storage="fp16", **M0)
    sim.set_plan(kernel, (32, 8, 5))
    orc = oracle.Sim(16, workloads.SEED, **M0)
    worst = np.zeros(5)
    for t in range(100):
        sim.step(1)
        orc.step(1)
        if (t + 1) % 10 == 0:
            worst = np.maximum(worst, _compare(sim, orc, TOL16, f"fp16 step {t + 1}", dtol=DTOL16))
    say(f"  fp16 worst rel errors rho/j/f = {worst[:3]}, deviation-relative drho/f = {worst[3:]}")


def test_plans_bit_identical():
    """Split, fused, staged and rows with different tiles and graph replay give
    the same bits."""
    lbf = require_gpu()
    L = 24
    say("plans L=24")
    states = []
    for kernel, tile, g in [("split", (0, 0, 0), 0), ("fused", (16, 16, 8), 0), ("fused", (32, 8, 24), 0),
                            ("fused", (32, 8, 5), 6), ("split", (0, 0, 0), 4), ("fused", (64, 4, 7), 0),
                            ("staged", (32, 8, 9), 0), ("staged", (16, 16, 24), 0), ("staged", (16, 8, 5), 4),
                            ("rows", (32, 8, 9), 0), ("rows", (16, 16, 24), 6), ("rows", (16, 8, 5), 0),
                            ("rows", (64, 4, 7), 0), ("rows", (64, 8, 7), 0), ("rows", (64, 8, 5), 4)]:
        sim = lbf.Sim(L, 11, **M0)
        sim.set_plan(kernel, tile, g)
        sim.step(13)
        states.append(sim.fields(f=True)["f"])
    for s in states[1:]:
        assert np.array_equal(s, states[0])


@pytest.mark.parametrize("L", [8, 24, 40])
def test_fp16_plans_bit_identical(L):
    """FP16 storage: split, the register-ring fused kernel and the rows
    staging (8-half chunks; 64 x 8 tiles with 512 threads too) give the same
    bits, with partial tiles (L = 40 against 32- and 64-wide tiles) and the
    source rows wrapping on L = 8."""
    lbf = require_gpu()
    say(f"fp16 plans L={L}")
    states = []
    for kernel, tile, g in [("split", (0, 0, 0), 0), ("fused", (32, 8, 7), 0), ("fused", (64, 4, 5), 3),
                            ("rows", (32, 8, 7), 0), ("rows", (64, 4, 9), 0), ("rows", (16, 16, 5), 4),
                            ("rows", (16, 8, 3), 0), ("rows", (64, 8, 5), 0), ("rows", (64, 8, 7), 3)]:
        sim = lbf.Sim(L, 21, storage="fp16", **M0)
        sim.set_plan(kernel, tile, g)
        sim.step(9)
        states.append(sim.fields(f=True)["f"])
    for s in states[1:]:
        assert np.array_equal(s, states[0])


def test_tuner_keeps_the_trajectory():
    """lb_tune steps the state through every candidate plan (split, fused,
    staged, rows; with and without graphs, sampling on): afterwards the
    state equals that of a handle stepped as often with the default plan,
    bit for bit, and the kept plan is one of the candidates."""
    lbf = require_gpu()
    L = 24
    say("tuner L=24")
    prm = dict(M0, sample_every=5)
    a = lbf.Sim(L, 31, **prm)
    best = a.tune(steps=4)
    assert best["kernel"] in (lbf.LB_KERNEL_SPLIT, lbf.LB_KERNEL_FUSED, lbf.LB_KERNEL_STAGED, lbf.LB_KERNEL_ROWS)
    assert a.plan() == best
    a.step(3)
    n = a.info()["step"]
    b = lbf.Sim(L, 31, **prm)
    b.step(n)
    assert np.array_equal(a.fields(f=True)["f"], b.fields(f=True)["f"])


def test_deterministic_repeat():
    lbf = require_gpu()
    say("repeat L=16")
    a = lbf.Sim(16, 1234, **M0)
    b = lbf.Sim(16, 1234, **M0)
    a.step(25)
    b.step(25)
    assert np.array_equal(a.fields(f=True)["f"], b.fields(f=True)["f"])
    c = lbf.Sim(16, 1235, **M0)
    c.step(25)
    assert not np.array_equal(a.fields()["rho"], c.fields()["rho"])


def test_batched_equals_plain():
    """Every replica of a batch of uneven sizes and parameters evolves bit for
    bit as it does alone."""
    lbf = require_gpu()
    say("batch vs plain")
    Ls = [8, 12, 5, 16, 9]
    seeds = [101, 102, 103, 104, 105]
    prms = [dict(M0, a=a) for a in (-0.02, 0.0, 0.02, 0.01, -0.01)]
    prms[2]["tau"] = 0.8
    prms[3]["kT"] = 2e-4
    bat = lbf.Sim.batch(Ls, seeds, prms)
    bat.step(17)
    for r, (L, sd, p) in enumerate(zip(Ls, seeds, prms)):
        one = lbf.Sim(L, sd, **p)
        one.step(17)
        fb = bat.fields(r, f=True)["f"]
        fo = one.fields(f=True)["f"]
        assert np.array_equal(fb, fo), f"replica {r}"


def test_unstable_flag_is_sticky():
    """A negative density (the positivity condition of Sec. III B) raises
    LB_EUNSTABLE at the next synchronisation, and stays raised."""
    lbf = require_gpu()
    say("unstable flag")
    L = 6
    f = workloads.random_populations(L, 1)
    f[:, 0] = -np.abs(f[:, 0])   # site 0 with rho < 0
    sim = lbf.Sim(L, 1, **M0)
    sim.step(1)
    sim.sync()
    with pytest.raises(lbf.LBError) as e:
        sim.set_populations(f)
        sim.step(1)
        sim.sync()
    assert e.value.code == lbf.LB_EUNSTABLE
    with pytest.raises(lbf.LBError):
        sim.sync()


def test_rows_plan_needs_multiple_of_four():
    """The rows staging copies 16-byte chunks, so a lattice edge that is not a
    multiple of 4 (FP32) or 8 (FP16) is refused with LB_EINVAL and the plan
    stays as it was."""
    lbf = require_gpu()
    sim = lbf.Sim(10, 1, **M0)
    before = sim.plan()
    with pytest.raises(lbf.LBError) as e:
        sim.set_plan("rows", (32, 8, 4))
    assert e.value.code == lbf.LB_EINVAL
    assert sim.plan() == before
    # FP16 chunks hold 8 halves: L = 12 passes the FP32 rule but not this one
    h = lbf.Sim(12, 1, storage="fp16", **M0)
    before = h.plan()
    with pytest.raises(lbf.LBError) as e:
        h.set_plan("rows", (32, 8, 4))
    assert e.value.code == lbf.LB_EINVAL
    assert h.plan() == before


@pytest.mark.parametrize("kernel", ["split", "rows"])
def test_separate_relaxation_times(kernel):
    """Bulk and ghost moments with their own relaxation times (tau_bulk = 1.3,
    tau_ghost = 0.6, tau = 0.8) against the oracle, every step of 30."""
    lbf = require_gpu()
    L = 12
    say(f"separate rates L={L} {kernel}")
    prm = dict(M0, tau=0.8, tau_bulk=1.3, tau_ghost=0.6, a=0.02, b=0.3)
    sim = lbf.Sim(L, 17, **prm)
    sim.set_plan(kernel, (16, 16, 5))
    orc = oracle.Sim(L, 17, **prm)
    for t in range(30):
        sim.step(1)
        orc.step(1)
        _compare(sim, orc, TOL32, f"step {t + 1}", dtol=DTOL32)


@pytest.mark.parametrize("kernel", ["split", "fused", "rows"])
def test_rest_state_is_exact_without_noise(kernel):
    """kT = 0 and a uniform density: every population is w_i rho_c at rest;
    the force, the noise and every moment beyond rho are zero, so the state
    stays exactly the rest state (stored deviations exactly zero)."""
    lbf = require_gpu()
    sim = lbf.Sim(12, 5, **dict(M0, kT=0.0, init_sigma=0.0))
    sim.set_plan(kernel, (16, 16, 5))
    sim.step(12)
    g = sim.fields(f=True)
    # every site identical (the stored deviations are exactly zero); the
    # exported rho sums w_i rho_c in FP64, equal to rho_c up to rounding
    assert np.array_equal(g["f"], np.broadcast_to(g["f"][:, :1], g["f"].shape))
    assert np.all(g["rho"] == g["rho"][0]) and abs(g["rho"][0] - M0["rho_c"]) < 1e-15
    assert not np.any(g["j"])


@pytest.mark.parametrize("name,prm", [
    ("no noise", dict(kT=0.0)),
    ("tau near 1/2", dict(tau=0.51)),
    ("no thermodynamic terms", dict(a=0.0, b=0.0, kappa=0.0)),
    ("strong noise", dict(kT=1e-3, tau=0.6)),
])
def test_degenerate_parameters(name, prm):
    """Edges of the parameter range against the oracle, every step of 10:
    deterministic dynamics (kT = 0), relaxation factor near -1 (tau = 0.51),
    the force reduced to the cancellation of the lattice pressure
    (a = b = kappa = 0), and ten times the workload's noise."""
    lbf = require_gpu()
    L = 12
    p = dict(M0, **prm)
    say(f"degenerate: {name}")
    sim = lbf.Sim(L, 23, **p)
    sim.set_plan("rows", (16, 16, 5))
    orc = oracle.Sim(L, 23, **p)
    for t in range(10):
        sim.step(1)
        orc.step(1)
        _compare(sim, orc, TOL32, f"{name} step {t + 1}", dtol=DTOL32)
