"""The three-dimensional structure factor (Sec. IV A, Eq. (G-comput)) at the
lattice sizes of the workloads, against the oracle's FFT of the same states:
64^3 and 256^3 (radix-2 passes over LDS tiles of 32 and 8 lines) and 512^3
(tiles of 4 lines).  Two kinds of state:

- the model's own fluctuating state after a few steps (every shell holds
  signal): shell sums within the rounding of the FP32 density snapshot the
  device transforms;
- a sum of plane waves of density seeded through the import path, among them
  the Nyquist planes kx = L/2 (the last column of the real-to-half-complex
  pass), ky = L/2, kz = L/2 and the corner (L/2, L/2, L/2): the shells that
  hold a seeded mode match the oracle, and the others must stay empty to
  1e-9 of the largest shell, which a wrong twiddle, index or tile edge in any
  pass would break.

The GPU transforms the FP32 snapshot of the density deviation, the oracle the
FP64 density exported from the same populations, so the per-shell agreement
is bounded by the FP32 rounding of the deviation (~1e-7 relative per mode).
"""
import numpy as np
import pytest

import workloads
from oracle import moments
from gpu_util import require_gpu, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

M0 = workloads.MODEL
# per shell: |g - o| <= RTOL |o| + ATOL max |o|
RTOL, ATOL = 2e-6, 1e-9


def _check_shells(g, ref, where):
    assert np.array_equal(g["modes"], ref["modes"]), where
    live = g["modes"] > 0
    assert np.allclose(g["k2"][live], ref["k2"][live], rtol=1e-12, atol=0), where
    assert np.allclose(g["lap"][live], ref["lap"][live], rtol=1e-12, atol=0), where
    o, x = ref["sum_C"], g["sum_C"]
    d = np.abs(x - o)
    big = np.max(np.abs(o))
    rel = d[live] / np.maximum(np.abs(o[live]), 1e-300)
    say(f"  {where}: {int(live.sum())} shells, max rel err {np.max(rel[np.abs(o[live]) > 1e-3 * big]):.2e}, "
        f"max abs err / max {np.max(d) / big:.2e}")
    bad = np.nonzero(d > RTOL * np.abs(o) + ATOL * big)[0]
    assert bad.size == 0, (where, bad[:8], x[bad[:8]], o[bad[:8]])


@pytest.mark.parametrize("L", [64, 256, 512])
def test_model_state_shell_sums(L):
    lbf = require_gpu()
    every = 3
    nsamp = 1 if L == 512 else 2
    say(f"sk3 model state L={L}, {nsamp} sample(s)")
    sim = lbf.Sim(L, 19, sample_every=every, sk3_stride=1, **dict(M0, a=0.02))
    acc = None
    for _ in range(nsamp):
        sim.step(every)
        rho = sim.fields(j=False)["rho"]
        C = moments.structure_factor_3d(moments.order_parameter(rho), L)
        del rho
        sh = moments.shell_average(C, L)
        del C
        if acc is None:
            acc = sh
        else:
            acc["sum_C"] = acc["sum_C"] + sh["sum_C"]
    g = sim.sk3()
    assert g["n_samples"] == nsamp
    _check_shells(g, acc, f"L={L}")


def _plane_wave_density(L, rng):
    """rho = 1 + sum_j A_j cos(2 pi m_j . r / L + phi_j) as flat [L^3]."""
    h = L // 2
    modes = [(1, 0, 0), (h, 0, 0), (0, h, 0), (0, 0, h), (h, h, h), (3, -5, 7), (h - 1, h - 2, -3),
             (-L // 4 + 1, 2, h), (17, 0, -h + 3), (h, 1, -1)]
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    rho = np.ones((L, L, L))
    for j, (mx, my, mz) in enumerate(modes):
        A = 1e-3 * (1 + 0.1 * j)
        rho += A * np.cos(2 * np.pi * (mx * x + my * y + mz * z) / L + rng.uniform(0, 2 * np.pi))
    return rho.reshape(-1)


@pytest.mark.parametrize("L", [256, 512])
def test_plane_waves_stay_in_their_shells(L):
    """Ideal lattice gas without noise (force off, kT = 0): a density plane
    wave stays at its wave vector under the linear step, so after one step
    the spectrum is the seeded modes (and second-order harmonics ~1e-6 of
    them)."""
    lbf = require_gpu()
    say(f"sk3 plane waves L={L}")
    rng = np.random.default_rng(L)
    rho = _plane_wave_density(L, rng)
    W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f = W[:, None] * rho[None, :]
    del rho
    sim = lbf.Sim(L, 3, sample_every=1, sk3_stride=1, force_off=True, kT=0.0, init_sigma=0.0, tau=1.0)
    sim.set_populations(f)
    del f
    sim.step(1)
    rho1 = sim.fields(j=False)["rho"]
    C = moments.structure_factor_3d(moments.order_parameter(rho1), L)
    del rho1
    ref = moments.shell_average(C, L)
    del C
    g = sim.sk3()
    assert g["n_samples"] == 1
    _check_shells(g, ref, f"plane waves L={L}")
    live = ref["modes"] > 0
    occupied = np.count_nonzero(ref["sum_C"][live] > 1e-6 * np.max(ref["sum_C"]))
    assert 5 <= occupied <= 20
