"""The paper's own model on D3Q19 (LB_EQ_PRESSURE: the non-ideal pressure in
the equilibrium, Sec. III A) on the GPU against its FP64 oracle
(oracle/d3q19_meq.py), through the C ABI: every step element by element
(L = 12 runs the rows kernel k_meq_staged, L = 7 and 10 the split passes),
the rows plan bit for bit against the split passes (every tile shape,
partial tiles, samples, graphs, batches, 256^3), conservation, the batch and
plan rules, and equilibrium statistics.  Tolerances are those of the force
model's parity tests (FP32 compute and storage against FP64: 1e-5 of the
field's largest value)."""
import numpy as np
import pytest

from oracle import d3q19_meq as OM
from gpu_util import rel_err, require_gpu, say

pytestmark = pytest.mark.gpu

PRM = dict(a=0.03, b=0.7, kappa=0.05, rho_c=1.0, kT=1e-4, tau=0.8, init_sigma=0.02)
TOL32 = 1e-5


def _compare(sim, orc, tol, where):
    g = sim.fields(rho=True, j=True, f=True)
    rho_o, j_o = orc.fields()
    e = (rel_err(g["rho"], rho_o), rel_err(g["j"], j_o), rel_err(g["f"], orc.f))
    if isinstance(tol, dict):
        ok = e[0] <= tol["rho"] and e[1] <= tol["j"] and e[2] <= tol["f"]
    else:
        ok = max(e) <= tol
    assert ok, f"{where}: rel errors rho/j/f = {e}"
    return e


@pytest.mark.parametrize("L", [12, 7, 10])
def test_every_step_against_oracle(L):
    lbf = require_gpu()
    say(f"eq-pressure model L={L}")
    sim = lbf.Sim(L, 40 + L, eq_pressure=True, **PRM)
    orc = OM.Sim(L, 40 + L, **PRM)
    worst = 0.0
    for t in range(30):
        sim.step(1)
        orc.step(1)
        worst = max(worst, max(_compare(sim, orc, TOL32, f"L={L} step {t + 1}")))
    say(f"  worst relative error {worst:.2e}")


def test_parameter_rules():
    """FP16 storage, LB_FORCE_OFF and separate relaxation times are refused
    with LB_EQ_PRESSURE: at rest the model keeps nearly all mass on the rest
    population (p0(rho_c) = 0), so the deviations from w_i rho_c that the
    storage holds are O(1), and binary16 would keep ~1e-3 of them."""
    lbf = require_gpu()
    for extra in (dict(storage="fp16"), dict(force_off=True), dict(tau_bulk=1.1), dict(tau_ghost=0.7)):
        with pytest.raises(lbf.LBError) as e:
            lbf.Sim(8, 1, eq_pressure=True, **dict(PRM, **extra))
        assert e.value.code == lbf.LB_EINVAL, extra


def test_exact_conservation_and_sampling():
    """No force: the total mass and momentum stay at their initial values
    (FP64 sums of FP32 fields) with the quartic term on, and the sample
    sums of a graph-replayed run equal those of direct launches."""
    lbf = require_gpu()
    L = 16
    a = lbf.Sim(L, 9, eq_pressure=True, sample_every=5, **dict(PRM, b=2.0))
    r0 = a.fields(rho=True, j=True)
    a.step(40)
    r1 = a.fields(rho=True, j=True)
    # FP32 rounding of the O(1) stored deviations random-walks: ~1e-7 per
    # site and step, so after 40 steps of 16^3 the mass moves by ~5e-9 of
    # itself (an FP32 emulation of the transforms; FP32-rounded weights in
    # the moment sums would instead drift by ~1e-7) and the momentum by
    # ~1e-7 of sum |j|
    assert abs(r1["rho"].sum() - r0["rho"].sum()) <= 5e-8 * r0["rho"].sum()
    assert np.abs(r1["j"].sum(axis=1) - r0["j"].sum(axis=1)).max() <= 1e-6 * np.abs(r1["j"]).sum()
    b = lbf.Sim(L, 9, eq_pressure=True, sample_every=5, **dict(PRM, b=2.0))
    b.set_plan("split", (0, 0, 0), 10)
    b.step(40)
    assert np.array_equal(a.fields(f=True)["f"], b.fields(f=True)["f"])
    ma, mb = a.moments(), b.moments()
    assert ma["n_samples"] == mb["n_samples"] == 8
    assert ma["levels"] == mb["levels"] and ma["mass"] == mb["mass"]


def test_batch_and_plan_rules():
    lbf = require_gpu()
    sim = lbf.Sim(8, 1, eq_pressure=True, **PRM)
    p = sim.plan()
    assert (p["kernel"], p["tile_x"], p["tile_y"]) == (lbf.LB_KERNEL_ROWS, 32, 8)
    for k, t in (("rows", (16, 8, 8)), ("fused", (16, 16, 8)), ("staged", (32, 8, 8))):
        with pytest.raises(lbf.LBError) as e:
            sim.set_plan(k, t)
        assert e.value.code == lbf.LB_EINVAL
    # the 16-byte row staging needs L a multiple of 4
    odd = lbf.Sim(10, 1, eq_pressure=True, **PRM)
    assert odd.plan()["kernel"] == lbf.LB_KERNEL_SPLIT
    with pytest.raises(lbf.LBError) as e:
        odd.set_plan("rows", (32, 8, 8))
    assert e.value.code == lbf.LB_EINVAL
    # a replica evolves in a batch exactly as alone
    Ls, seeds = [8, 12, 6], [4, 5, 6]
    prms = [dict(PRM, eq_pressure=True, a=a) for a in (0.02, 0.03, 0.05)]
    bat = lbf.Sim.batch(Ls, seeds, prms)
    bat.step(9)
    for r in range(3):
        one = lbf.Sim(Ls[r], seeds[r], **prms[r])
        one.step(9)
        assert np.array_equal(bat.fields(r, f=True)["f"], one.fields(f=True)["f"])
    # the model must be the same for every replica of a batch
    with pytest.raises(lbf.LBError) as e:
        lbf.Sim.batch([8, 8], [1, 2], [dict(PRM, eq_pressure=True), dict(PRM)])
    assert e.value.code == lbf.LB_EINVAL


def _run(lbf, L, seed, plan, steps, sample_every=3, prm=PRM):
    sim = lbf.Sim(L, seed, eq_pressure=True, sample_every=sample_every, **prm)
    sim.set_plan(*plan)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("L,tile", [(12, (32, 8, 5)), (20, (64, 4, 7)), (16, (16, 16, 16)), (24, (64, 4, 24)),
                                    (36, (16, 16, 9)), (8, (64, 4, 3)), (24, (64, 8, 5)), (40, (32, 16, 13)),
                                    (68, (64, 8, 23)), (4, (32, 8, 4)), (4, (64, 8, 1))])
def test_rows_plan_equals_split(L, tile):
    """k_meq_staged (full and partial tiles, slabs that do not divide L)
    against the density and collide passes: the same populations and FP64
    sample sums bit for bit, with a sample (written by the step kernel)
    every 3 steps and with graphs."""
    lbf = require_gpu()
    say(f"eq-pressure rows {tile} against split, L={L}")
    prm = dict(PRM, b=2.0)
    a = _run(lbf, L, 60 + L, ("split", (0, 0, 0)), 17, prm=prm)
    b = _run(lbf, L, 60 + L, ("rows", tile), 17, prm=prm)
    c = _run(lbf, L, 60 + L, ("rows", tile, 6), 17, prm=prm)
    fa = a.fields(f=True)["f"]
    for o in (b, c):
        assert np.array_equal(o.fields(f=True)["f"], fa)
        ma, mo = a.moments(), o.moments()
        assert ma["n_samples"] == mo["n_samples"] == 5
        assert ma["mass"] == mo["mass"] and ma["levels"] == mo["levels"]
        assert np.array_equal(ma["momentum"], mo["momentum"]) and np.array_equal(ma["sk"], mo["sk"])


def test_rows_plan_batch():
    """A batch on the rows plan (tiles of every replica in one launch): each
    replica as it evolves alone on the split passes."""
    lbf = require_gpu()
    Ls, seeds = [8, 12, 16, 20], [4, 5, 6, 7]
    prms = [dict(PRM, eq_pressure=True, a=a) for a in (0.02, 0.03, 0.05, 0.04)]
    bat = lbf.Sim.batch(Ls, seeds, prms)
    assert bat.plan()["kernel"] == lbf.LB_KERNEL_ROWS
    bat.step(9)
    for r in range(4):
        one = lbf.Sim(Ls[r], seeds[r], **prms[r])
        one.set_plan("split", (0, 0, 0))
        one.step(9)
        assert np.array_equal(bat.fields(r, f=True)["f"], one.fields(f=True)["f"]), r


def test_rows_plan_256():
    """256^3 at the bench's parameters: the default plan (rows, 64 x 8 tiles
    in eight slabs) and the split passes give bit-identical FP64 sample sums
    (mass, momentum, block levels, axis S(k)) after every step."""
    lbf = require_gpu()
    import workloads
    L, steps = 256, 3
    prm = dict(workloads.MODEL)
    say(f"eq-pressure {L}^3: default plan against split, {steps} steps, sample every step")
    a = lbf.Sim(L, workloads.SEED, eq_pressure=True, sample_every=1, **prm)
    p = a.plan()
    assert (p["kernel"], p["tile_x"], p["tile_y"], p["tile_z"]) == (lbf.LB_KERNEL_ROWS, 64, 8, 32)
    a.step(steps)
    ma = a.moments()
    del a
    b = lbf.Sim(L, workloads.SEED, eq_pressure=True, sample_every=1, **prm)
    b.set_plan("split", (0, 0, 0))
    b.step(steps)
    mb = b.moments()
    del b
    assert ma["n_samples"] == mb["n_samples"] == steps
    assert ma["mass"] == mb["mass"] and ma["levels"] == mb["levels"]
    assert np.array_equal(ma["momentum"], mb["momentum"]) and np.array_equal(ma["sk"], mb["sk"])


@pytest.mark.timeout(900)
def test_256_against_oracle():
    """256^3 at the bench's parameters, the default plan (the rows kernel on
    64 x 8 tiles in eight slabs): the first step against the FP64 oracle
    over the whole lattice (under a minute of host time)."""
    lbf = require_gpu()
    import workloads
    L = 256
    prm = dict(workloads.MODEL)
    say(f"eq-pressure {L}^3, default plan, 1 step")
    sim = lbf.Sim(L, workloads.SEED, eq_pressure=True, **prm)
    p = sim.plan()
    assert (p["kernel"], p["tile_x"], p["tile_y"]) == (lbf.LB_KERNEL_ROWS, 64, 8)
    sim.step(1)
    got = sim.fields(rho=True, j=True, f=True)
    del sim
    say("  oracle 256^3, 1 step (under a minute)")
    orc = OM.Sim(L, workloads.SEED, **prm)
    orc.step(1)
    rho_o, j_o = orc.fields()
    e = (rel_err(got["rho"], rho_o), rel_err(got["j"], j_o), rel_err(got["f"], orc.f))
    say(f"  rel errors rho/j/f {e}")
    assert max(e) <= TOL32


def test_unstable_sound_speed_is_flagged():
    """c_s^2 >= 1/2 leaves the noise covariance without a real factor: with
    kT > 0 the step raises the sticky LB_EUNSTABLE."""
    lbf = require_gpu()
    sim = lbf.Sim(8, 1, eq_pressure=True, **dict(PRM, a=0.6, b=0.0))
    sim.step(1)
    with pytest.raises(lbf.LBError) as e:
        sim.sync()
    assert e.value.code == lbf.LB_EUNSTABLE


def test_equilibrium_statistics_32():
    """b = 0, a = 0.05, kappa = 1e-3: <|rho_k|^2>/N = kT / (a + kappa lam(k))
    (the compressibility of the Landau free energy, Sec. II A, with the
    lattice Laplacian's symbol lam) at every wave vector, and
    <|j_k|^2>/N = rho kT per component (Eq. (vel-correl)); 32^3, 2000 steps
    discarded, 400 samples every 10 steps.  Averaged over all modes the
    ratios are within 2% (the oracle on 8^3 gives 0.99-1.005 in every band
    of k); over the 32 modes of smallest k within 10% (a sound mode there
    decorrelates over ~250 steps: ~16 independent samples each)."""
    lbf = require_gpu()
    L = 32
    prm = dict(a=0.05, b=0.0, kappa=1e-3, rho_c=1.0, kT=1e-4, tau=0.8, init_sigma=0.0)
    sim = lbf.Sim(L, 77, eq_pressure=True, **prm)
    sim.set_plan("split", (0, 0, 0), 10)
    sim.step(2000)
    S = np.zeros((L, L, L))
    J = np.zeros((L, L, L))
    n = 400
    for _ in range(n):
        sim.step(10)
        g = sim.fields(rho=True, j=True)
        rk = np.fft.fftn((g["rho"] - g["rho"].mean()).reshape(L, L, L))
        S += np.abs(rk) ** 2 / L ** 3
        for a in range(3):
            J += np.abs(np.fft.fftn(g["j"][a].reshape(L, L, L))) ** 2 / (3 * L ** 3)
    S /= n
    J /= n
    k = 2 * np.pi * np.fft.fftfreq(L)
    K = np.meshgrid(k, k, k, indexing="ij")  # axes (z, y, x) of the reshaped field
    lam = np.zeros((L, L, L))
    for i in range(19):
        c = OM.C[i]
        lam += 6 * OM.W[i] * (1 - np.cos(K[2] * c[0] + K[1] * c[1] + K[0] * c[2]))
    ratio = S / (prm["kT"] / (prm["a"] + prm["kappa"] * lam))
    ratio[0, 0, 0] = np.nan
    J[0, 0, 0] = np.nan
    low = (lam > 0) & (lam <= np.sort(lam[lam > 0].ravel())[31])
    say(f"  S/theory: all k {np.nanmean(ratio):.4f}, smallest 32 modes {np.nanmean(ratio[low]):.4f}; "
        f"<|j_k|^2>/(N kT) {np.nanmean(J) / prm['kT']:.4f}")
    assert abs(np.nanmean(ratio) - 1) < 0.02
    assert abs(np.nanmean(ratio[low]) - 1) < 0.10
    assert abs(np.nanmean(J) / prm["kT"] - 1) < 0.02
