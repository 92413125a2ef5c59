"""The largest lattice the library takes, L = 1024 (2^30 sites; 163 GB of
FP32 populations, 82 GB of FP16), where every 32-bit site, plane and byte
offset of the kernels is at its limit.  No oracle runs at this size; the
checks are properties that hold at any size:

- the FP64 sample sums (mass, momentum, every block level's moment sums and
  the axis structure factor, sampled after every step) of the default rows
  plan and of the split kernels agree bit for bit: the two paths index the
  lattice with different code (64-bit site indices and neighbour tables in
  the split kernels; tile origins, 32-bit plane offsets and row-staged
  chunks in the rows kernel), so an offset that wraps in one of them shows;
- mass is conserved from the initial state to FP32 (FP16) rounding."""
import numpy as np
import pytest

import workloads
from gpu_util import require_gpu, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

L = 1024


def _run(lbf, storage, plan, steps):
    sim = lbf.Sim(L, workloads.SEED, storage=storage, sample_every=1, **workloads.MODEL)
    if plan is not None:
        sim.set_plan(*plan)
    m0 = sim.moments()["mass"]
    sim.step(steps)
    m = sim.moments()
    p = sim.plan()
    del sim
    return m0, m, p


@pytest.mark.parametrize("storage,tol", [("fp16", 2e-6), ("fp32", 2e-7)])
def test_max_lattice_plans_agree(storage, tol):
    lbf = require_gpu()
    steps = 2
    say(f"{L}^3 {storage}: default plan, {steps} steps, sample every step")
    m0, a, pa = _run(lbf, storage, None, steps)
    # both storages default to 64 x 8 rows tiles on large lattices; FP32
    # samples on its 64 x 4 snapshot table (sample every step here)
    assert (pa["kernel"], pa["tile_x"], pa["tile_y"]) == (lbf.LB_KERNEL_ROWS, 64, 8)
    say(f"  {pa}; mass {m0!r} -> {a['mass']!r}")
    say(f"{L}^3 {storage}: split kernels")
    _, b, _ = _run(lbf, storage, ("split", (0, 0, 0)), steps)
    assert a["n_samples"] == b["n_samples"] == steps
    assert a["mass"] == b["mass"]
    assert np.array_equal(a["momentum"], b["momentum"])
    assert len(a["levels"]) == len(b["levels"]) == 10
    for la, lb in zip(a["levels"], b["levels"]):
        assert la == lb, (la["Lb"], la, lb)
    assert np.array_equal(a["sk"], b["sk"])
    # mass: the lattice holds 2^30 rho_c; the populations round to FP32 or
    # FP16 deviations on each store, the sums are FP64
    assert abs(a["mass"] - m0) <= tol * m0
    assert abs(m0 / L ** 3 - workloads.MODEL["rho_c"]) < 1e-4
