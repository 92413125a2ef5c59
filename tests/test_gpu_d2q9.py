"""The paper's own D2Q9 model on the GPU (lb2_*) against the D2Q9 oracle
(oracle/d2q9.py): initial state, every step of 100 (FP32 against FP64),
exact conservation, the spectra, and the equilibrium statistics the paper
checks (Eq. (CMF) for the density, Eq. (vel-correl) for the momentum, its
longitudinal and transverse parts as in the paper's equilibration figure)."""
import numpy as np
import pytest

from oracle import d2q9 as D
from oracle import moments
from gpu_util import rel_err, require_gpu, say

pytestmark = pytest.mark.gpu

PRM = dict(a=0.03, b=0.5, kappa=0.01, rho_c=1.0, kT=1e-5, tau=0.8, init_sigma=0.02)


def _sim(lbf, L, seed, **prm):
    return lbf.Sim2D(L, seed, **prm)


@pytest.mark.parametrize("L", [16, 12, 7])
def test_every_step_against_oracle(L):
    lbf = require_gpu()
    say(f"d2q9 parity L={L}")
    g = _sim(lbf, L, 3, **PRM)
    o = D.Sim(L, 3, **PRM)
    st = g.fields(f=True)
    assert rel_err(st["f"], o.f) < 1e-6
    worst = 0.0
    for t in range(100):
        g.step(1)
        o.step(1)
        st = g.fields(f=True)
        rho_o, j_o = o.fields()
        e = (rel_err(st["rho"], rho_o), rel_err(st["j"], j_o), rel_err(st["f"], o.f))
        worst = max(worst, max(e))
        assert max(e) < 1e-5, (t + 1, e)
    say(f"  worst relative error {worst:.2e}")


@pytest.mark.parametrize("L,steps", [(100, 10), (38, 10), (256, 10), (2048, 2), (4, 20), (5, 20)])
def test_tiled_step_against_oracle(L, steps):
    """Lattices of several 64 x 4 tiles with partial ones at the edges (100:
    two tiles across x, the second 36 wide; 38: one partial tile across x
    and a last row of tiles 2 high), the paper's 256^2 (256 tiles dealt to
    the XCDs in runs), the largest lattice, 2048^2 (16384 tiles), and the
    smallest, 4^2 and 5^2 (one tile whose halo wraps onto the lattice):
    every step against the oracle."""
    lbf = require_gpu()
    say(f"d2q9 tiled parity L={L}, {steps} steps")
    g = _sim(lbf, L, 11, **PRM)
    o = D.Sim(L, 11, **PRM)
    worst = 0.0
    for t in range(steps):
        g.step(1)
        o.step(1)
        st = g.fields(f=True)
        rho_o, j_o = o.fields()
        e = (rel_err(st["rho"], rho_o), rel_err(st["j"], j_o), rel_err(st["f"], o.f))
        worst = max(worst, max(e))
        assert max(e) < 1e-5, (L, t + 1, e)
    say(f"  worst relative error {worst:.2e}")


def test_mass_and_momentum_conserved():
    lbf = require_gpu()
    L = 32
    g = _sim(lbf, L, 5, **dict(PRM, b=2.0, init_sigma=0.05))
    s0 = g.fields()
    g.step(300)
    s1 = g.fields()
    N = L * L
    assert abs(s1["rho"].sum() - s0["rho"].sum()) / N < 1e-7
    assert np.max(np.abs(s1["j"].sum(axis=1) - s0["j"].sum(axis=1))) / N < 1e-9


def test_import_export_round_trip():
    lbf = require_gpu()
    L = 10
    g = _sim(lbf, L, 1, **PRM)
    rng = np.random.default_rng(2)
    f = D.equilibrium(1.0 + 0.02 * rng.standard_normal(L * L), 0.01 * rng.standard_normal((2, L * L)), L, PRM)
    g.set_populations(f)
    assert rel_err(g.fields(f=True)["f"], f) < 1e-7
    o = D.Sim(L, 1, **PRM)
    o.f = f.copy()
    g.step(5)
    o.step(5)
    assert rel_err(g.fields(f=True)["f"], o.f) < 1e-5


def _oracle_spectra(rho, j, L):
    N = L * L
    dr = np.fft.fft2((rho - 1.0).reshape(L, L))
    jx = np.fft.fft2(j[0].reshape(L, L))
    jy = np.fft.fft2(j[1].reshape(L, L))
    m = moments.folded_modes(L).astype(float)   # wave numbers in (-L/2, L/2]
    my, mx = np.meshgrid(m, m, indexing="ij")
    kn = np.sqrt(mx * mx + my * my)
    with np.errstate(invalid="ignore", divide="ignore"):
        hx = np.where(kn > 0, mx / kn, 0.0)
        hy = np.where(kn > 0, my / kn, 0.0)
    par = hx * jx + hy * jy
    perp = -hy * jx + hx * jy
    return {"S": np.abs(dr) ** 2 / N, "Jx": np.abs(jx) ** 2 / N, "Jy": np.abs(jy) ** 2 / N,
            "Jpar": np.abs(par) ** 2 / N, "Jperp": np.abs(perp) ** 2 / N}


@pytest.mark.parametrize("L", [12, 16, 64, 256, 512, 1024, 2048])
def test_spectra_against_oracle_transform(L):
    """The GPU's spectra of its own states equal numpy's FFT of the exported
    fields (the GPU sums the same FP32 state in FP64): direct transforms for
    L = 12, radix-2 FFTs for the powers of two, up to 2048^2."""
    lbf = require_gpu()
    g = _sim(lbf, L, 8, sample_every=3, **PRM)
    acc = None
    for _ in range(5):
        g.step(3)
        st = g.fields()
        sp = _oracle_spectra(st["rho"], st["j"], L)
        acc = sp if acc is None else {k: acc[k] + sp[k] for k in acc}
    got = g.spectra()
    assert got["n_samples"] == 5
    for k in ("S", "Jx", "Jy", "Jpar", "Jperp"):
        scale = np.max(np.abs(acc[k][1:])) if k != "S" else np.max(np.abs(acc[k].reshape(-1)[1:]))
        d = np.abs(got[k] - acc[k]).reshape(-1)[1:]
        assert np.max(d) <= 1e-9 * scale, (k, np.max(d) / scale)
    g.reset_spectra()
    assert g.spectra()["n_samples"] == 0


def test_equilibrium_statistics_64():
    """b = 0, a = 0.05, kappa = 1e-3, kT = 1e-5, tau = 0.8 on 64^2: averaged
    over all k != 0, S(k) (a + kappa k_lat^2)/kT and <|j_a,k|^2>/(N kT) (x, y,
    longitudinal, transverse) are 1 within 2% (the paper's equilibration
    check), and the first axis modes within 5%."""
    lbf = require_gpu()
    L = 64
    prm = dict(a=0.05, b=0.0, kappa=1e-3, rho_c=1.0, kT=1e-5, tau=0.8, init_sigma=0.0)
    say("d2q9 statistics 64^2")
    g = _sim(lbf, L, 11, sample_every=20, **prm)
    g.step(4000)
    g.reset_spectra()
    g.step(100000)
    sp = g.spectra()
    n = sp["n_samples"]
    m = np.fft.fftfreq(L) * L
    ky, kx = np.meshgrid(2 * np.pi * m / L, 2 * np.pi * m / L, indexing="ij")
    lap = 6 * ((1 / 9) * (4 - 2 * np.cos(kx) - 2 * np.cos(ky)) + (1 / 36) * (4 - 2 * np.cos(kx + ky) - 2 * np.cos(kx - ky)))
    th = prm["kT"] / (prm["a"] + prm["kappa"] * lap)
    rS = (sp["S"] / n / th).reshape(-1)[1:]
    say(f"  S/theory mean {rS.mean():.4f}; axis {np.round((sp['S'] / n / th)[0, 1:6], 3)}")
    assert abs(rS.mean() - 1) < 0.02
    assert np.all(np.abs((sp["S"] / n / th)[0, 1:4] - 1) < 0.05)
    for k in ("Jx", "Jy", "Jpar", "Jperp"):
        r = (sp[k] / n / prm["kT"]).reshape(-1)[1:]
        say(f"  {k}/kT mean {r.mean():.4f}")
        assert abs(r.mean() - 1) < 0.02, k


@pytest.mark.parametrize("L", [48, 64])
def test_batch_replicas_equal_single_handles(L):
    """Replicas of one L in one handle (lb2_create_batch), each with its own
    parameters and seed: fields and spectra bit for bit those of the same
    replica alone (direct DFT spectra at L = 48, FFTs at L = 64), and one
    replica against the oracle."""
    lbf = require_gpu()
    say(f"d2q9 batch L={L}")
    seeds = [21, 22, 23, 24]
    prms = [dict(PRM, sample_every=5), dict(PRM, a=0.05, sample_every=5), dict(PRM, kT=2e-5, sample_every=5),
            dict(PRM, tau=0.7, b=0.2, sample_every=5)]
    bat = lbf.Sim2D.batch(L, seeds, prms)
    bat.step(23)
    for r, (sd, p) in enumerate(zip(seeds, prms)):
        one = lbf.Sim2D(L, sd, **p)
        one.step(23)
        fb, fo = bat.fields(f=True, replica=r), one.fields(f=True)
        for k in ("rho", "j", "f"):
            assert np.array_equal(fb[k], fo[k]), (r, k)
        sb, so = bat.spectra(r), one.spectra()
        assert sb["n_samples"] == so["n_samples"] == 4
        for k in ("S", "Jx", "Jy", "Jpar", "Jperp"):
            assert np.array_equal(sb[k], so[k]), (r, k)
    o = D.Sim(L, seeds[2], **{k: v for k, v in prms[2].items() if k != "sample_every"})
    o.step(23)
    assert rel_err(bat.fields(f=True, replica=2)["f"], o.f) < 1e-5
    # imports land in their own replica
    f1 = bat.fields(f=True, replica=1)["f"]
    bat.set_populations(bat.fields(f=True, replica=3)["f"], replica=1)
    assert np.array_equal(bat.fields(f=True, replica=1)["f"], bat.fields(f=True, replica=3)["f"])
    assert not np.array_equal(f1, bat.fields(f=True, replica=1)["f"])
